"""Pins of the oracle's Hodge-Laplacian solver (oracle/hodge.py; Sec. 7.2,
eq:hodge-laplace, eq:augmented-lagrangian, thm:augmented-lagrangian-hl;
no GPU).

* the exterior derivative D: d o d = 0 (curl grad = 0 and div curl = 0
  through the three derivative matrices) and D^T M_k D = the independently
  assembled stiffness of X^{k-1} (quadrature of the Piola-mapped
  derivatives; for k = 3 this pins the DG mass 1 / |det J| as well);
* the mixed matrix and its preconditioner against the theorem: with the
  exact weighted Riesz maps, every generalized eigenvalue is -1 or
  mu gamma / (mu gamma + 1), nu gamma / (nu gamma + 1) with mu, nu the
  nonzero eigenvalues of the two d-problems (the Fichera corner has no
  harmonic 1-, 2- or 3-forms), checked eigenvalue by eigenvalue;
* MINRES: the dense solution, monotone preconditioned residuals, and the
  solution and iteration count of scipy's MINRES (an independent
  implementation) on the same system;
* the paper's p = 1 rows of tab:hodge-fichera: the Schwarz solvers are
  exact at p = 1 (the Whitney group is the whole space), so the MINRES
  counts follow from the theorem's spectrum and do not depend on the mesh
  -- 6 iterations at gamma = 1 and 3 at gamma = 1e3 for CG_1 x Ned_1 and
  Ned_1 x RT_1, 5 and 3 for RT_1 x DG_0, reproduced exactly on a
  Freudenthal mesh of the Fichera corner.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.hodge import (HodgeLaplacian, cell_volume_ratio, derivative_matrix, derivative_reference,
                          divergence_reference_dg, minres, theorem_spectrum)
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


@pytest.mark.parametrize("p", [1, 2, 3, pytest.param(4, marks=pytest.mark.slow)])
def test_derivatives_form_a_complex(p):
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=5)
    tops = [Topology(X, C, element(3, f, p)) for f in ("CG", "Ned", "RT")]
    D1 = derivative_matrix(tops[0], tops[1], derivative_reference(1, p))
    D2 = derivative_matrix(tops[1], tops[2], derivative_reference(2, p))
    assert abs(D2 @ D1).max() < 1e-10
    H3 = HodgeLaplacian(X, C, 3, p, exact=True)
    assert H3.top0.n_dofs == tops[2].n_dofs
    assert abs(H3.D @ D2).max() < 1e-10
    # on the vertex functions and the Whitney edge functions, grad is the
    # signed incidence (lem:basis-contains-whitney): +1 at the larger vertex
    t0, t1 = tops[0], tops[1]
    wj = t1.kinds[1].index("W")
    for e, (a, b) in enumerate(t1.ent_tuples[1]):
        row = D1[t1.offset[1] + e * t1.N[1] + wj, :t0.n_vertices].toarray().ravel()
        want = np.zeros(t0.n_vertices)
        want[a], want[b] = -1.0, 1.0
        assert np.abs(row - want).max() < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_derivative_reproduces_the_stiffness(k, p):
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=7)
    H = HodgeLaplacian(X, C, k, p, exact=True)
    K0 = (H.D.T @ H.M1 @ H.D).toarray()
    K0ref = assemble(H.top0, all_cell_matrices(H.el0, H.top0, alpha=1.0, beta=0.0)).toarray()
    assert np.abs(K0 - K0ref).max() <= 1e-12 * np.abs(K0ref).max()


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("gamma", [1.0, pytest.param(10.0, marks=pytest.mark.slow), 1e3])
def test_preconditioned_spectrum_is_the_theorems(k, gamma):
    X, C = fichera_mesh(2, jitter=0.1, seed=3)
    H = HodgeLaplacian(X, C, k, 1 if gamma != 10.0 else 2, gamma=gamma, exact=True)
    B = sla.block_diag(H.R0.toarray(), H.R1.toarray())
    lam = np.sort(sla.eigh(H.A.toarray(), B, eigvals_only=True))
    th = theorem_spectrum(H)
    assert len(th) == len(lam)
    assert np.abs(lam - th).max() <= 1e-8
    assert np.sum(np.abs(lam + 1) < 1e-9) >= H.n0


@pytest.mark.parametrize("k", [1, 2, 3])
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


@pytest.mark.parametrize("cx,k", [("CG_Ned", 1), ("Ned_RT", 2), ("RT_DG", 3)])
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


@pytest.mark.parametrize("p", [1, 2, 3])
def test_dg_block(p):
    """X^3 = DG_{p-1}: the per-cell volume ratio and diagonal mass, and Gauss'
    theorem through D.  Of the orthonormal Dubiner functions only the
    constant one has a nonzero mean, int psi_hat_0 = sqrt(|T_hat|), and the
    3-form pullback gives int_T psi_0 = sign(det J_T) sqrt(|T_hat|).  The
    Whitney function of a facet has unit flux through that facet and none
    through the others, so int_T div = +-1 on each cell of the facet, with
    opposite signs on the two cells of an interior facet; the DG
    coefficients u = D sigma must reproduce that (up to one global sign,
    the orientation of the reference cell)."""
    from oracle.simplex import EQ_VERTICES
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=9)
    H = HodgeLaplacian(X, C, 3, p, exact=True)
    E = EQ_VERTICES[3]
    vol_hat = abs(np.linalg.det((E[1:] - E[0]).T)) / 6.0
    Cs = np.sort(C, axis=1)
    sgn = np.array([np.sign(np.linalg.det((X[c][1:] - X[c][0]).T)) for c in Cs])
    vol = np.array([abs(np.linalg.det((X[c][1:] - X[c][0]).T)) / 6.0 for c in Cs])
    assert np.allclose(H.detJ * vol_hat, vol, rtol=1e-13)
    assert np.allclose(H.M1.diagonal(), np.repeat(1.0 / H.detJ, H.ndg))
    # the integral of each DG function over its cell
    integ = np.zeros(H.n1)
    integ[::H.ndg] = sgn * np.sqrt(vol_hat)
    t = H.top0
    wj = t.kinds[2].index("W")
    for f in range(0, len(t.ent_tuples[2]), 7):
        sig = np.zeros(H.n0)
        sig[t.offset[2] + f * t.N[2] + wj] = 1.0
        per_cell = (integ * (H.D @ sig)).reshape(-1, H.ndg).sum(axis=1)
        nz = np.flatnonzero(np.abs(per_cell) > 1e-12)
        assert 1 <= len(nz) <= 2
        assert np.allclose(np.abs(per_cell[nz]), 1.0, atol=1e-12)
        if len(nz) == 2:
            assert abs(per_cell[nz].sum()) < 1e-12
