"""Pins of the oracle's Hodge-Laplacian solver (oracle/hodge.py; Sec. 7.2,
eq:hodge-laplace, eq:augmented-lagrangian, thm:augmented-lagrangian-hl;
no GPU).

* the exterior derivative D: d o d = 0 (curl grad = 0 through the two
  derivative matrices) and D^T M_k D = the independently assembled
  stiffness of X^{k-1} (quadrature of the Piola-mapped derivatives);
* the mixed matrix and its preconditioner against the theorem: with the
  exact weighted Riesz maps, every generalized eigenvalue is -1 or
  mu gamma / (mu gamma + 1), nu gamma / (nu gamma + 1) with mu, nu the
  nonzero eigenvalues of the two d-problems (the Fichera corner has no
  harmonic 1- or 2-forms), checked eigenvalue by eigenvalue;
* MINRES: the dense solution, monotone preconditioned residuals, and the
  solution and iteration count of scipy's MINRES (an independent
  implementation) on the same system;
* the paper's p = 1 rows of tab:hodge-fichera: the Schwarz solvers are
  exact at p = 1 (the Whitney group is the whole space), so the MINRES
  counts follow from the theorem's spectrum and do not depend on the mesh
  -- 6 iterations at gamma = 1 and 3 at gamma = 1e3 for CG_1 x Ned_1 and
  Ned_1 x RT_1, reproduced exactly on a Freudenthal mesh of the Fichera
  corner.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.hodge import HodgeLaplacian, derivative_matrix, derivative_reference, minres, theorem_spectrum
from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble
from paper_2506_17406_amd.workloads import fichera_mesh, kuhn_mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_hodge_fichera.csv")


def _paper_rows():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            cx, p, dofs, s1, f1, s3, f3 = line.strip().split(",")
            out[(cx, int(p))] = (int(dofs), int(s1), int(f1), int(s3), int(f3))
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_derivatives_form_a_complex(p):
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=5)
    tops = [Topology(X, C, element(3, f, p)) for f in ("CG", "Ned", "RT")]
    D1 = derivative_matrix(tops[0], tops[1], derivative_reference(1, p))
    D2 = derivative_matrix(tops[1], tops[2], derivative_reference(2, p))
    assert abs(D2 @ D1).max() < 1e-10
    # on the vertex functions and the Whitney edge functions, grad is the
    # signed incidence (lem:basis-contains-whitney): +1 at the larger vertex
    t0, t1 = tops[0], tops[1]
    wj = t1.kinds[1].index("W")
    for e, (a, b) in enumerate(t1.ent_tuples[1]):
        row = D1[t1.offset[1] + e * t1.N[1] + wj, :t0.n_vertices].toarray().ravel()
        want = np.zeros(t0.n_vertices)
        want[a], want[b] = -1.0, 1.0
        assert np.abs(row - want).max() < 1e-12


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_derivative_reproduces_the_stiffness(k, p):
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=7)
    H = HodgeLaplacian(X, C, k, p, exact=True)
    K0 = (H.D.T @ H.M1 @ H.D).toarray()
    K0ref = assemble(H.top0, all_cell_matrices(H.el0, H.top0, alpha=1.0, beta=0.0)).toarray()
    assert np.abs(K0 - K0ref).max() <= 1e-12 * np.abs(K0ref).max()


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("gamma", [1.0, 10.0, 1e3])
def test_preconditioned_spectrum_is_the_theorems(k, gamma):
    X, C = fichera_mesh(2, jitter=0.1, seed=3)
    H = HodgeLaplacian(X, C, k, 1 if gamma != 10.0 else 2, gamma=gamma, exact=True)
    B = sla.block_diag(H.R0.toarray(), H.R1.toarray())
    lam = np.sort(sla.eigh(H.A.toarray(), B, eigvals_only=True))
    th = theorem_spectrum(H)
    assert len(th) == len(lam)
    assert np.abs(lam - th).max() <= 1e-8
    assert np.sum(np.abs(lam + 1) < 1e-9) >= H.n0


@pytest.mark.parametrize("k", [1, 2])
def test_minres_against_dense_and_scipy(k):
    X, C = fichera_mesh(2, jitter=0.1, seed=11)
    H = HodgeLaplacian(X, C, k, 2, gamma=10.0)
    b = H.rhs(np.random.default_rng(1).uniform(-1, 1, H.n1))
    x, info = minres(lambda v: H.A @ v, H.apply_P, b, rtol=1e-12, maxit=500)
    xd = np.linalg.solve(H.A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-14)
    # scipy's MINRES with the same preconditioner (as a LinearOperator)
    n = len(b)
    P = spla.LinearOperator((n, n), matvec=H.apply_P)
    xs, code = spla.minres(H.A, b, M=P, rtol=1e-10, maxiter=500)
    assert code == 0
    assert np.linalg.norm(xs - xd) <= 1e-7 * np.linalg.norm(xd)
    x8, info8 = minres(lambda v: H.A @ v, H.apply_P, b, rtol=1e-10, maxit=500)
    assert np.linalg.norm(x8 - xs) <= 1e-7 * np.linalg.norm(xd)


@pytest.mark.parametrize("cx,k", [("CG_Ned", 1), ("Ned_RT", 2)])
@pytest.mark.parametrize("gamma", [1.0, 1e3])
def test_paper_p1_minres_counts(cx, k, gamma):
    rows = _paper_rows()
    _, s1, f1, s3, f3 = rows[(cx, 1)]
    want = s1 if gamma == 1.0 else s3
    X, C = fichera_mesh(4)
    for dec in ("paper", "paper-full"):
        H = HodgeLaplacian(X, C, k, 1, gamma=gamma, decomposition=dec)
        b = H.rhs(np.random.default_rng(3).uniform(-1, 1, H.n1))
        _, info = minres(lambda v: H.A @ v, H.apply_P, b, rtol=1e-8)
        assert info["iterations"] == want, (dec, info["iterations"], want)
