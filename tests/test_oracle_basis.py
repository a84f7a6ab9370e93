"""Pins of the oracle's reference construction against facts the paper and
the mathematics fix (no GPU).

* orthonormal polynomials and quadrature: closed-form simplex moments;
* SplitMix64: published output for seed 0;
* space and bubble dimensions: closed forms (eq:bubble-trace-dim-counts);
* lem:ref-element-matrix-properties: K_II = [I 0; 0 0], K_IG = 0,
  M_II = diag(Lambda, I), M_{I^II, G} = 0;
* lem:basis-contains-whitney: the Whitney basis functions are the textbook
  barycentric Whitney forms;
* lem:trace-basis-eigenfunctions: traces of type-I functions are the
  eigenfunctions;
* lem:d-preserves-basis-functions: the local discrete gradient is the
  Whitney incidence plus the identity on type-I -> type-II dofs;
* d o d = 0 on the local sequence CG_p -> Ned_p -> RT_p.
"""
from itertools import combinations
from math import factorial

import numpy as np
import pytest

from oracle.element import (FORM, eigenbasis, element, entity_map, make_space,
                            reference_matrices, space_dim, trace)
from oracle.simplex import EQ_VERTICES, PolyBasis, quadrature, simplex_volume, splitmix64_stream


def bary(d, x):
    V = EQ_VERTICES[d]
    A = np.vstack([V.T, np.ones(d + 1)])
    return np.linalg.solve(A, np.vstack([x.T, np.ones(x.shape[0])])).T


@pytest.mark.parametrize("d", [1, 2, 3])
def test_quadrature_barycentric_moments(d):
    # int_T lambda^a = a! d! |T| / (|a| + d)!  (closed form)
    x, w = quadrature(d, 6)
    lam = bary(d, x)
    rng = np.random.default_rng(0)
    for _ in range(10):
        a = rng.integers(0, 4, size=d + 1)
        exact = np.prod([factorial(int(ai)) for ai in a]) * factorial(d) * simplex_volume(d) \
            / factorial(int(a.sum()) + d)
        assert np.isclose(np.sum(w * np.prod(lam ** a, axis=1)), exact, rtol=1e-13, atol=0)


@pytest.mark.parametrize("d,p", [(1, 10), (2, 10), (3, 8)])
def test_dubiner_orthonormal(d, p):
    B = PolyBasis(d, p)
    x, w = quadrature(d, p + 2)
    V = B.values(x)
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(B.n)).max() < 1e-13
    # spans P_p: exact reproduction of a random polynomial in barycentrics
    lam = bary(d, x)
    f = lam[:, 0] ** p + 3 * lam[:, -1] * lam[:, 0] ** (p - 1)
    c = V.T @ (w * f)
    assert np.abs(V @ c - f).max() < 1e-12


def test_gradients_match_finite_differences():
    B = PolyBasis(3, 6)
    x = np.array([[0.1, 0.05, -0.1], [-0.3, -0.2, -0.1]])
    g = B.gradients(x)
    h = 1e-6
    fd = np.stack([(B.values(x + h * e) - B.values(x - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    assert np.abs(g - fd).max() < 1e-7 * np.abs(g).max()


def test_splitmix64_published_value():
    # SplitMix64 (Steele, Lea, Flood 2014) with state 0: first output
    # 0xe220a8397b1dcdaf; the stream yields its top 53 bits scaled to [0,1).
    g = splitmix64_stream(0)
    assert next(g) == (0xE220A8397B1DCDAF >> 11) / 2.0 ** 53


@pytest.mark.parametrize("l,fam", [(2, "Ned"), (3, "Ned"), (2, "RT"), (3, "RT"), (2, "NedTwo"), (3, "NedTwo"),
                                   (3, "BDM")])
@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_space_dimensions(l, fam, p):
    assert make_space(l, fam, p).m == space_dim(l, fam, p)


def _bubble_counts(p):
    """Appendix-style closed forms for the type-I counts N^k_S."""
    return {
        ("CG", 1): p - 1, ("CG", 2): (p - 1) * (p - 2) // 2, ("CG", 3): (p - 1) * (p - 2) * (p - 3) // 6,
        ("Ned", 2): (p - 1) * (p + 2) // 2, ("Ned", 3): (p - 1) * (p - 2) * (2 * p + 3) // 6,
        ("NedTwo", 2): (p - 1) * (p + 2) // 2, ("NedTwo", 3): (p - 1) * (p - 2) * (2 * p + 3) // 6,
        ("RT", 3): (p - 1) * (p * p + 4 * p + 6) // 6,
    }


@pytest.mark.parametrize("p", [2, 3, 4, pytest.param(6, marks=pytest.mark.slow)])
def test_type_one_counts_and_kernel(p):
    for (fam, l), n in _bubble_counts(p).items():
        eb = eigenbasis(l, fam, p)
        assert eb.N == n, (fam, l, p)
        if eb.N == 0:
            continue
        # eq:bubble-trace-dim-counts: dim bubbles = N^k + N^{k-1}
        assert len(eb.mu_all) == eb.N + eb.n_ker if eb.N else True
        # eq:ref-eval-problem-x: (d psi_i, d psi_j) = delta, (psi_i, psi_j) = lambda_i delta
        x, w = quadrature(l, p + 2)
        v = eb.values(x)
        dv = eb.dvalues(x)
        G = np.einsum("q,qci,qcj->ij", w, dv, dv)
        M = np.einsum("q,qci,qcj->ij", w, v, v)
        assert np.abs(G - np.eye(eb.N)).max() < 1e-11
        assert np.abs(M - np.diag(eb.lam)).max() < 1e-11 * max(1, eb.lam.max())


def _blocks(el):
    M, K = reference_matrices(el)
    I = el.interior()
    kinds = np.array([di.kind for di in el.dofs])
    I1, I2 = I & (kinds == "I"), I & (kinds == "II")
    return M, K, I, ~I, I1, I2


@pytest.mark.parametrize("d,fam,p", [(2, "CG", 4), (2, "CG", 7), (3, "CG", 3), (3, "CG", 6),
                                     (3, "Ned", 2), (3, "Ned", 4), pytest.param(3, "Ned", 6, marks=pytest.mark.slow),
                                     (3, "RT", 2), (3, "RT", 4), pytest.param(3, "RT", 6, marks=pytest.mark.slow),
                                     (2, "Ned", 3), (2, "Ned", 6), (2, "RT", 3), (2, "RT", 6),
                                     (3, "NedTwo", 2), (3, "NedTwo", 4), (3, "BDM", 2), (3, "BDM", 4)])
def test_reference_matrix_structure(d, fam, p):
    """lem:ref-element-matrix-properties."""
    el = element(d, fam, p)
    M, K, I, G, I1, I2 = _blocks(el)
    eb = eigenbasis(d, fam, p)
    if not I.any():
        return
    KII = K[np.ix_(I, I)]
    expect = np.zeros_like(KII)
    n1 = int(I1.sum())
    expect[:n1, :n1] = np.eye(n1)
    assert np.abs(KII - expect).max() < 1e-11
    assert np.abs(K[np.ix_(I, G)]).max() < 1e-12
    MII = M[np.ix_(I, I)]
    assert np.abs(MII - np.diag(np.r_[eb.lam, np.ones(int(I2.sum()))])).max() < 1e-11
    if I2.any():
        assert np.abs(M[np.ix_(I2, G)]).max() < 1e-12
    # diagonal scaling of the interior blocks gives condition number one and
    # exactly one nonzero per interior row (Sec. 4.3)
    assert np.count_nonzero(np.abs(KII + MII) > 1e-10, axis=1).max() == 1


def _whitney(d, k, verts, x):
    lam = bary(d, x)
    V = EQ_VERTICES[d]
    A = np.vstack([V.T, np.ones(d + 1)])
    grad = np.linalg.inv(A)[:, :d]          # rows: grad lambda_m
    if k == 0:
        return lam[:, verts[0]][:, None]
    if k == 1:
        a, b = verts
        return lam[:, a, None] * grad[b] - lam[:, b, None] * grad[a]
    a, b, c = verts
    cr = lambda i, j: np.cross(grad[i], grad[j])
    return 2 * (lam[:, a, None] * cr(b, c) + lam[:, b, None] * cr(c, a) + lam[:, c, None] * cr(a, b))


@pytest.mark.parametrize("d,fam,p", [(2, "CG", 3), (3, "CG", 4), (3, "Ned", 1), (3, "Ned", 4),
                                     (3, "RT", 1), (3, "RT", 4)])
def test_basis_contains_whitney_forms(d, fam, p):
    """lem:basis-contains-whitney, against the barycentric formulas."""
    el = element(d, fam, p)
    rng = np.random.default_rng(1)
    lam = rng.dirichlet(np.ones(d + 1), size=20)
    x = lam @ EQ_VERTICES[d]
    vals, _ = el.tabulate(x)
    k = el.k
    for i, di in enumerate(el.dofs):
        if di.kind == "W":
            w = _whitney(d, k, di.verts, x)
            assert np.abs(vals[:, :, i] - w).max() < 1e-12, (fam, di.verts)


@pytest.mark.parametrize("d,fam,p", [(3, "CG", 5), (3, "Ned", 4), (3, "RT", 4), (2, "CG", 5)])
def test_traces_are_eigenfunctions(d, fam, p):
    """lem:trace-basis-eigenfunctions: tr_S phi^I_{S,j} = psi_{S,j} and
    tr_S phi^II_{S,n} = d_S psi^{k-1}_{S,n} on every subentity."""
    el = element(d, fam, p)
    k = el.k
    lower = {1: "CG", 2: "NedTwo"}.get(k)
    for i, di in enumerate(el.dofs):
        l = di.entity_dim
        if di.kind == "W" or l == 0:
            continue
        o, A, y0 = entity_map(d, di.verts)
        y, _ = quadrature(l, 3)
        x = o + (y - y0) @ A.T
        vals, _ = el.tabulate(x)
        tr = trace(k, A, vals)[:, :, i]
        if di.kind == "I":
            ref = eigenbasis(l, fam, p).values(y)[:, :, di.j]
        else:
            ref = eigenbasis(l, lower, p).dvalues(y)[:, :, di.j]
        assert np.abs(tr - ref).max() < 1e-10 * max(1.0, np.abs(ref).max()), (fam, di.verts, di.kind, di.j)


def _project(el_target, field_coef, c):
    """Coefficients in P_p^c of a field already given in P_p^c coefficients."""
    return field_coef


def _derivative_coeffs(el, target_space_l):
    """Primal (P_p^c') coefficients of d phi_j for the basis of el."""
    x, w = quadrature(el.d, el.p + 2)
    _, dv = el.tabulate(x)
    poly = el.space.poly
    V = poly.values(x)
    return np.einsum("q,qcj,qn->cnj", w, dv, V).reshape(-1, el.n)


@pytest.mark.parametrize("p", [1, 2, 3, pytest.param(5, marks=pytest.mark.slow)])
def test_local_discrete_gradient_structure(p):
    """lem:d-preserves-basis-functions: the Ned_p dofs of grad phi^CG_j are the
    Whitney incidence (vertex -> +-1 on its edges) plus the identity from CG
    type-I to Ned type-II dofs of the same entity."""
    cg, ned = element(3, "CG", p), element(3, "Ned", p)
    Gloc = ned.L @ _derivative_coeffs(cg, 3)
    expect = np.zeros_like(Gloc)
    for j, dj in enumerate(cg.dofs):
        for i, di in enumerate(ned.dofs):
            if dj.entity_dim == 0 and di.kind == "W":
                a, b = di.verts
                if dj.verts[0] == b:
                    expect[i, j] = 1.0
                elif dj.verts[0] == a:
                    expect[i, j] = -1.0
            elif dj.entity_dim > 0 and di.kind == "II" and di.verts == dj.verts and di.j == dj.j:
                expect[i, j] = 1.0
    assert np.abs(Gloc - expect).max() < 1e-11


@pytest.mark.parametrize("p", [1, 3, 4])
def test_local_sequence_d_of_d_is_zero(p):
    """d o d = 0 through the dof maps: curl (grad CG) = 0 in RT dofs and the
    RT coefficients of curl Ned have zero divergence."""
    cg, ned, rt = element(3, "CG", p), element(3, "Ned", p), element(3, "RT", p)
    G = ned.L @ _derivative_coeffs(cg, 3)
    C = rt.L @ _derivative_coeffs(ned, 3)
    assert np.abs(C @ G).max() < 1e-10 * np.abs(C).max()
    # the RT function with coefficients C[:, j] equals curl phi^Ned_j
    x, w = quadrature(3, p + 2)
    vr, dvr = rt.tabulate(x)
    _, curl = ned.tabulate(x)
    assert np.abs(np.einsum("qci,ij->qcj", vr, C) - curl).max() < 1e-10 * np.abs(curl).max()
    assert np.abs(np.einsum("qci,ij->qcj", dvr, C)).max() < 1e-10 * np.abs(dvr).max()
