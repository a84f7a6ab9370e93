"""Pins of the oracle parts that other checks rely on (no GPU).

* The stacked form: A_T = sum_q w_{T,q} R_q (the reference stack and the
  geometric weights of the Piola maps, eq:pullback-3d-def) against the
  definition, quadrature of the pulled-back basis on the physical cell
  (eq:weak-form), on random and strongly anisotropic cells and for several
  (alpha, beta).  A transposed Jacobian, a swapped component pair, a missing
  1/det or an alpha/beta mix-up fails it.
* The eigen-cluster convention (reading R2): the canonical basis of a
  cluster of equal eigenvalues does not depend on the orthonormal basis of
  the eigenspace that the eigensolver returned (random rotations and
  reflections inside every cluster leave it unchanged).
* The gap census behind R2: for every (subsimplex dimension, family, p)
  that the elements up to p = 10 use, the clusters are separated by far
  more than the cluster tolerance, the spread inside a cluster is at
  rounding level, and the probe matrices are well conditioned.
"""
import numpy as np
import pytest

from oracle.element import (TAU, bubble_eigenproblem, canonical_clusters, cluster_bounds, cluster_census,
                            eigenbasis, element)
from oracle.operator import cell_matrix, cell_weights, reference_stack
from oracle.simplex import EQ_VERTICES, quadrature

COEFFS = [(1.0, 1.0), (1e3, 1.0), (1e-3, 1.0), (1.0, 0.25)]


def _cells(d, rng, n=20):
    """n random cells (a scaled unit simplex with every vertex moved by up to
    30% of its size, random placement and size) and one strongly anisotropic
    cell (aspect ratio 100)."""
    base = np.vstack([np.zeros(d), np.eye(d)])
    out = []
    for _ in range(n):
        h = rng.uniform(0.05, 2.0)
        X = h * (base + rng.uniform(-0.3, 0.3, size=base.shape)) + rng.uniform(-5, 5, size=d)
        out.append(X)
    aniso = base.copy()
    aniso[1:] *= np.array([1.0, 0.01, 0.1][:d])[:, None] if d == 3 else np.array([1.0, 0.01])[:, None]
    out.append(aniso + 0.5)
    return out


@pytest.mark.parametrize("d,fam,p", [(2, f, p) for f in ("CG", "Ned", "RT") for p in range(1, 7)]
                         + [(3, f, p) if p <= (4 if f == "CG" else 3) else pytest.param(3, f, p, marks=pytest.mark.slow)
                            for f in ("CG", "Ned", "RT") for p in range(1, 7)]
                         + [(3, f, p) if p <= 3 else pytest.param(3, f, p, marks=pytest.mark.slow)
                            for f in ("NedTwo", "BDM") for p in range(1, 5)])
def test_stacked_form_equals_cell_quadrature(d, fam, p):
    el = element(d, fam, p)
    R = reference_stack(el)
    xq, wq = quadrature(el.d, el.p + 2)
    tab = (wq,) + el.tabulate(xq)
    rng = np.random.default_rng(1000 + 10 * p + d)
    worst = 0.0
    for X in _cells(d, rng):
        for alpha, beta in COEFFS:
            A = cell_matrix(el, X, alpha, beta, tab)
            w = cell_weights(el, X, alpha, beta)
            S = np.tensordot(w, R, axes=1)
            worst = max(worst, np.abs(S - A).max() / np.abs(A).max())
    assert worst < 1e-13, worst


def test_stacked_form_detects_swapped_coefficients():
    """Control: the comparison above is sensitive to an alpha/beta swap."""
    el = element(3, "Ned", 2)
    R = reference_stack(el)
    X = _cells(3, np.random.default_rng(3), 1)[0]
    A = cell_matrix(el, X, 1e3, 1.0)
    S = np.tensordot(cell_weights(el, X, 1.0, 1e3), R, axes=1)
    assert np.abs(S - A).max() / np.abs(A).max() > 1e-2


def _random_cluster_rotation(bounds, n, rng):
    Q = np.zeros((n, n))
    for i, j in bounds:
        m = j - i
        G, _ = np.linalg.qr(rng.standard_normal((m, m)))
        G = G @ np.diag(rng.choice([-1.0, 1.0], size=m))
        Q[i:j, i:j] = G
    return Q


@pytest.mark.parametrize("l,fam,p", [(2, "CG", 4), (2, "CG", 7), (3, "CG", 6), pytest.param(3, "CG", 8, marks=pytest.mark.slow),
                                     (2, "Ned", 5), (3, "Ned", 4), pytest.param(3, "Ned", 5, marks=pytest.mark.slow),
                                     (3, "RT", 4), pytest.param(3, "RT", 5, marks=pytest.mark.slow), (2, "NedTwo", 4),
                                     (3, "NedTwo", 4), (2, "RT", 5), (3, "BDM", 4)])
def test_cluster_canonicalisation_is_basis_invariant(l, fam, p):
    sp, Bb, K, mu, Vec, n_ker = bubble_eigenproblem(l, fam, p)
    mu_keep, W = mu[n_ker:], Vec[:, n_ker:]
    bounds = cluster_bounds(mu_keep)
    assert max(j - i for i, j in bounds) >= 2, "case has no degenerate cluster"
    W0, mu0, _ = canonical_clusters(l, sp, Bb, K, mu_keep, W)
    rng = np.random.default_rng(7 + p)
    for _ in range(3):
        Q = _random_cluster_rotation(bounds, W.shape[1], rng)
        W1, mu1, _ = canonical_clusters(l, sp, Bb, K, mu_keep, W @ Q)
        F0, F1 = Bb @ W0, Bb @ W1
        assert np.abs(F1 - F0).max() <= 1e-12 * np.abs(F0).max()
        np.testing.assert_allclose(mu1, mu0, rtol=1e-11)
        # the rotation was not the identity on the eigensolver's basis
        assert np.abs(Bb @ (W @ Q) - F0).max() > 1e-3 * np.abs(F0).max()
    # the element's eigenbasis is this canonical basis, scaled by mu^{-1/2}
    eb = eigenbasis(l, fam, p)
    assert np.abs(eb.Psi - F0 / np.sqrt(mu0)).max() <= 1e-12 * np.abs(eb.Psi).max()


def _census_cases(p):
    """(l, family, degree) of every eigenbasis the degree-p elements build:
    type-I bubbles of CG/Ned/RT, the CG and NedTwo type-II families and the
    kernel family CG_{p+1} of NedTwo_p."""
    out = [(l, "CG", p) for l in (1, 2, 3)] + [(l, "Ned", p) for l in (2, 3)]
    out += [(l, "NedTwo", p) for l in (2, 3)] + [(3, "RT", p)] + [(l, "CG", p + 1) for l in (1, 2, 3)]
    return out


@pytest.mark.slow
@pytest.mark.parametrize("p", list(range(2, 9)) + [pytest.param(p, marks=pytest.mark.heavy) for p in (9, 10)])
def test_eigen_gap_census(p):
    """Clusters are at least 100 TAU apart, equal to rounding inside, and
    probed by matrices of condition < 1e6 (observed: gaps >= 2.5e-5, spread
    <= 5e-14, cond(Y) <= 3.3e3 up to p = 10)."""
    for l, fam, q in _census_cases(p):
        c = cluster_census(eigenbasis(l, fam, q))
        assert c["min_gap"] > 100 * TAU, (l, fam, q, c)
        assert c["max_spread"] < 1e-11, (l, fam, q, c)
        assert c["max_cond"] < 1e6, (l, fam, q, c)
        assert c["max_size"] <= (2 if l == 2 else 3 if l == 3 else 1), (l, fam, q, c)
