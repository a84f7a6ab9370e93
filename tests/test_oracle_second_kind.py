"""Pins of the oracle's second-kind solve spaces NedTwo_p (H(curl)) and
BDM_p (H(div)) (eq:second-kind-def; no GPU).

The paper builds their dofs like the first kind's, with the type-II
functionals taken from the next-lower space of the second-kind sequence
CG_{p+1} -> NedTwo_p and NedTwo_{p+1} -> BDM_p (the remark after
eq:hdiv-dofs).  Checked against what the mathematics fixes:

* lem:basis-contains-whitney: the Whitney 1- and 2-forms (barycentric
  formulas) are basis functions;
* lem:trace-basis-eigenfunctions: the type-II traces are the derivatives of
  the CG_{p+1} (edges) and NedTwo_{p+1} (faces) eigenfunctions;
* lem:d-preserves-basis-functions: grad CG_{p+1} in NedTwo_p dofs and curl
  NedTwo_{p+1} in BDM_p dofs are the signed incidences plus the identity
  from type-I to type-II, the gradients have zero curl image, and div curl
  = 0 (the sequence is exact);
* Galerkin energy rates h^p on manufactured fields, and Schwarz
  preconditioners that are SPD, solve to the dense solution and keep their
  counts bounded in p.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401

from oracle.element import eigenbasis, element, entity_map, trace
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble, functional_load
from oracle.pcg import pcg
from oracle.precond import AdditiveSchwarz, HybridSchwarz
from oracle.simplex import EQ_VERTICES, quadrature
from paper_2506_17406_amd.workloads import kuhn_mesh


def _bary(x):
    V = EQ_VERTICES[3]
    A = np.vstack([V.T, np.ones(4)])
    lam = np.linalg.solve(A, np.vstack([x.T, np.ones(len(x))])).T
    return lam, np.linalg.inv(A)[:, :3]


@pytest.mark.parametrize("fam", ["NedTwo", "BDM"])
@pytest.mark.parametrize("p", [1, 3])
def test_basis_contains_whitney_forms(fam, p):
    el = element(3, fam, p)
    x = np.random.default_rng(1).dirichlet(np.ones(4), size=20) @ EQ_VERTICES[3]
    lam, g = _bary(x)
    vals, _ = el.tabulate(x)
    nW = 0
    for i, di in enumerate(el.dofs):
        if di.kind != "W":
            continue
        nW += 1
        if fam == "NedTwo":
            a, b = di.verts
            w = lam[:, a, None] * g[b] - lam[:, b, None] * g[a]
        else:
            a, b, c = di.verts
            cr = lambda i, j: np.cross(g[i], g[j])
            w = 2 * (lam[:, a, None] * cr(b, c) + lam[:, b, None] * cr(c, a) + lam[:, c, None] * cr(a, b))
        assert np.abs(vals[:, :, i] - w).max() < 1e-12
    assert nW == (6 if fam == "NedTwo" else 4)


@pytest.mark.parametrize("fam,p", [("NedTwo", 2), ("NedTwo", 4), ("BDM", 2), ("BDM", 3)])
def test_type_two_traces(fam, p):
    el = element(3, fam, p)
    lower, l_type = ("CG", 1) if fam == "NedTwo" else ("NedTwo", 2)
    for i, di in enumerate(el.dofs):
        if di.kind != "II" or di.entity_dim != l_type:
            continue
        o, A, y0 = entity_map(3, di.verts)
        y, _ = quadrature(l_type, 3)
        x = o + (y - y0) @ A.T
        vals, _ = el.tabulate(x)
        tr = trace(el.k, A, vals)[:, :, i]
        ref = eigenbasis(l_type, lower, p + 1).dvalues(y)[:, :, di.j]
        assert np.abs(tr - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def _derivative_coeffs(el, target):
    """Coefficients of d phi_j (phi_j the basis of el) in the orthonormal
    Dubiner basis of the target's space (exact: the derivative of a degree
    p + 1 field has degree p)."""
    x, w = quadrature(el.d, el.p + 2)
    _, dv = el.tabulate(x)
    V = target.space.poly.values(x)
    return np.einsum("q,qcj,qn->cnj", w, dv, V).reshape(-1, el.n)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_gradient_of_cg_p_plus_one(p):
    cg, el = element(3, "CG", p + 1), element(3, "NedTwo", p)
    G = el.L @ _derivative_coeffs(cg, el)
    expect = np.zeros_like(G)
    for j, dj in enumerate(cg.dofs):
        for i, di in enumerate(el.dofs):
            if dj.entity_dim == 0 and di.kind == "W":
                a, b = di.verts
                expect[i, j] = 1.0 if dj.verts[0] == b else (-1.0 if dj.verts[0] == a else 0.0)
            elif dj.entity_dim > 0 and di.kind == "II" and di.verts == dj.verts and di.j == dj.j:
                expect[i, j] = 1.0
    assert np.abs(G - expect).max() < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_curl_of_nedtwo_p_plus_one(p):
    """curl NedTwo_{p+1} in BDM_p dofs: the Whitney edge function to the
    Whitney functions of its faces with the sign of Stokes' theorem, a
    type-I function to the type-II function of the same entity and index, a
    gradient (type-II) to zero; and div of the image is zero."""
    nt, el = element(3, "NedTwo", p + 1), element(3, "BDM", p)
    C = el.L @ _derivative_coeffs(nt, el)
    for j, dj in enumerate(nt.dofs):
        col = C[:, j]
        if dj.kind == "II":
            assert np.abs(col).max() < 1e-10
        elif dj.kind == "I":
            want = np.array([1.0 if (di.kind == "II" and di.verts == dj.verts and di.j == dj.j) else 0.0
                             for di in el.dofs])
            assert np.abs(col - want).max() < 1e-10
        else:
            a0, b0 = dj.verts
            for i, di in enumerate(el.dofs):
                if di.kind == "W" and set(dj.verts) <= set(di.verts):
                    a, b, c = di.verts
                    assert abs(col[i] - (-1.0 if (a0, b0) == (a, c) else 1.0)) < 1e-10
                elif di.kind == "W":
                    assert abs(col[i]) < 1e-10
    x, _ = quadrature(3, p + 2)
    _, dv = el.tabulate(x)
    assert np.abs(np.einsum("qci,ij->qcj", dv, C)).max() < 1e-9 * max(1.0, np.abs(dv).max())


def _fields(fam):
    if fam == "NedTwo":
        u = lambda x: np.stack([np.sin(x[:, 1]), np.sin(x[:, 2]), np.sin(x[:, 0])], axis=1) * 3
        du = lambda x: -np.stack([np.cos(x[:, 2]), np.cos(x[:, 0]), np.cos(x[:, 1])], axis=1) * 3
    else:
        u = lambda x: np.stack([np.sin(2 * x[:, 0]) * x[:, 1], np.cos(x[:, 2]) * x[:, 0], np.exp(x[:, 1])], axis=1)
        du = lambda x: (2 * np.cos(2 * x[:, 0]) * x[:, 1])[:, None]
    return u, du


@pytest.mark.slow
@pytest.mark.parametrize("fam", ["NedTwo", "BDM"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_energy_convergence(fam, p):
    """Energy error decays like h^p: the derivative part dominates (curl
    NedTwo_p and div BDM_p are polynomials of degree p - 1)."""
    u, du = _fields(fam)
    errs = []
    for n in (2, 4):
        X, C = kuhn_mesh(n, 3, jitter=0.1, seed=5)
        top = Topology(X, C, element(3, fam, p))
        A = assemble(top, all_cell_matrices(top.el, top))
        b, energy = functional_load(top.el, top, u, du)
        x = sp.linalg.spsolve(A.tocsc(), b)
        errs.append(np.sqrt(max(energy - b @ x, 0.0)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p - 0.35, (errs, rate)


CASES = [("NedTwo", d) for d in ("paper", "paper-full", "vertex", "hiptmair")] + \
        [("BDM", d) for d in ("paper", "paper-full", "vertex", "typeI", "typeI-full", "hiptmair")]


@pytest.mark.parametrize("fam,dec", CASES)
def test_schwarz_spd_and_solves(fam, dec):
    X, C = kuhn_mesh(1, 3, jitter=0.1, seed=3)
    top = Topology(X, C, element(3, fam, 2))
    A = assemble(top, all_cell_matrices(top.el, top, alpha=1.3, beta=0.7))
    P = AdditiveSchwarz(A, top, fam, dec)
    Pm = np.stack([P.apply(e) for e in np.eye(top.n_dofs)], axis=1)
    assert np.abs(Pm - Pm.T).max() < 1e-11 * np.abs(Pm).max()
    assert np.linalg.eigvalsh(0.5 * (Pm + Pm.T)).min() > 0
    b = np.random.default_rng(2).uniform(-1, 1, top.n_dofs)
    x, _ = pcg(lambda v: A @ v, HybridSchwarz(A, top, fam, decomposition=dec).apply, b, rtol=1e-13)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.slow
@pytest.mark.parametrize("fam", ["NedTwo", "BDM"])
def test_hybrid_counts_bounded_in_p(fam):
    """Observed on the jittered 2-per-edge Kuhn mesh: NedTwo 10, 14, 16, 17
    and BDM 13, 16, 17, 18 iterations at p = 1..4 (rtol 1e-8)."""
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=3)
    its = []
    for p in (1, 2, 3, 4):
        top = Topology(X, C, element(3, fam, p))
        A = assemble(top, all_cell_matrices(top.el, top))
        b = np.random.default_rng(1).uniform(-1, 1, top.n_dofs)
        _, info = pcg(lambda v: A @ v, HybridSchwarz(A, top, fam).apply, b, rtol=1e-8)
        its.append(info["iterations"])
    assert max(its) <= 22 and its[-1] - its[1] <= 5, its
