"""Pins of the oracle's symmetric multiplicative hybrid preconditioner
(Sec. 7.1, eq:generic-subspace-splitting-mult).

* The paper's own numbers (tests/golden/paper_hybrid_level0.csv, from the
  result tables tab:hgrad-unit-cube, tab:hcurl-unit-cube and
  tab:hdiv-unit-cube): on the level-0 mesh (unit cube, 3 cells per edge) the
  dof counts are exact, PCG to 1e-8 in the preconditioned norm (reading R18)
  takes the printed number of iterations within 2, and the Lanczos condition
  estimate is within 6% of the printed one (the paper's right-hand side is an
  unspecified random vector).  Dropping the weights, the coarse space, or the
  multiplicative order moves the estimate by far more than that.
* The comparators (tests/golden/paper_vertex_star_level0.csv and
  paper_comparators_level0.csv, the same tables): PAFW(0)(X^k_Gamma) +
  J(X^k_I) and the full vertex stars PAFW(0)(X^k) for every space; for
  H(curl) PH(X^0, X^{1,I}), PH(X^0_Gamma, X^1_Gamma) + J(X^1_I) and
  PH(X^0, X^1); for H(div) PAFW(1)(X^2), PH(X^{1,I}_Gamma, X^{2,I}_Gamma) +
  J(X^2_I) and PH(X^{1,I}, X^{2,I}), and the standard Hiptmair-Toselli
  PH(X^1_Gamma, X^2_Gamma) + J(X^2_I) and PH(X^1, X^2) with the
  epsilon-regularised NedTwo potentials -- to the same bars.  These pin the
  star lists (with or without the cell interiors, type-I or every kind),
  the full potentials, the empty interior group of the full forms and the
  same weights and sweep.
* Algebra: the sweep is symmetric and positive definite, and its error
  propagator I - B A is the product of the group propagators
  (I - rho_m^{-1} B_m A) in the order 1, 2, 3, 2, 1.
* Weights: the 10-step Lanczos extremes lie inside the exact spectrum of the
  preconditioned subspace operator (Cauchy interlacing) and the largest is
  within 5% of the exact largest eigenvalue.
"""
import csv
import os

import numpy as np
import pytest

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble
from oracle.pcg import lanczos_condest, pcg
from oracle.precond import (SEED_INTERFACE, SEED_INTERIOR, HybridSchwarz, curl_potential_patches, patch_lists,
                            potential_patches, subspace_extremes, vertex_star_lists)
from paper_2506_17406_amd.workloads import kuhn_mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_hybrid_level0.csv")
GOLDEN_VSTAR = os.path.join(os.path.dirname(__file__), "golden", "paper_vertex_star_level0.csv")
GOLDEN_COMP = os.path.join(os.path.dirname(__file__), "golden", "paper_comparators_level0.csv")


def golden_rows():
    with open(GOLDEN) as f:
        rows = [r for r in csv.reader(l for l in f if not l.startswith("#"))]
    return [(r[0], int(r[1]), int(r[2]), float(r[3]), int(r[4]), float(r[5])) for r in rows]


def golden_vstar_rows():
    rows = []
    for path in (GOLDEN_VSTAR, GOLDEN_COMP):
        with open(path) as f:
            rows += [r for r in csv.reader(l for l in f if not l.startswith("#"))]
    return [(r[0], r[1], int(r[2]), int(r[3]), float(r[4]), int(r[5]), float(r[6])) for r in rows]


def build(fam, p, n=3, alpha=1.0, jitter=0.0):
    X, C = kuhn_mesh(n, 3, jitter=jitter, seed=3)
    top = Topology(X, C, element(3, fam, p))
    A = assemble(top, all_cell_matrices(top.el, top, alpha=alpha))
    return top, A


@pytest.mark.parametrize("row", golden_rows(), ids=lambda r: f"{r[0]}{r[1]}-alpha{r[3]:g}")
def test_paper_level0_iterations_and_condest(row):
    fam, p, dofs, alpha, its, cond = row
    top, A = build(fam, p, alpha=alpha)
    assert top.n_dofs == dofs
    H = HybridSchwarz(A, top, fam)
    b = np.random.default_rng(5).uniform(-1.0, 1.0, top.n_dofs)
    _, info = pcg(lambda v: A @ v, H.apply, b, rtol=1e-8, maxit=300, norm="preconditioned")
    assert abs(info["iterations"] - its) <= 2
    assert abs(lanczos_condest(info["alphas"], info["betas"]) / cond - 1.0) <= 0.06


def _slow_above(rows, key, limit):
    """The rows whose degree exceeds limit as slow cases (the cheapest degree
    of every space, decomposition and coefficient always runs)."""
    return [pytest.param(r, marks=pytest.mark.slow) if key(r) > limit else r for r in rows]


@pytest.mark.parametrize("row", _slow_above(golden_vstar_rows(), lambda r: r[2], 2),
                         ids=lambda r: f"{r[0]}{r[2]}-{r[1]}-alpha{r[4]:g}")
def test_paper_level0_comparator_solvers(row):
    fam, form, p, dofs, alpha, its, cond = row
    top, A = build(fam, p, alpha=alpha)
    assert top.n_dofs == dofs
    H = HybridSchwarz(A, top, fam, decomposition=form)
    if form.endswith("full"):
        assert len(H.add.I) == 0 and len(H.Gamma) == top.n_dofs
    b = np.random.default_rng(5).uniform(-1.0, 1.0, top.n_dofs)
    _, info = pcg(lambda v: A @ v, H.apply, b, rtol=1e-8, maxit=300, norm="preconditioned")
    assert abs(info["iterations"] - its) <= 2
    assert abs(lanczos_condest(info["alphas"], info["betas"]) / cond - 1.0) <= 0.06


GOLDEN_L1 = os.path.join(os.path.dirname(__file__), "golden", "paper_level1_gmg_coarse.csv")


def golden_l1_rows():
    with open(GOLDEN_L1) as f:
        rows = [r for r in csv.reader(l for l in f if not l.startswith("#"))]
    return [(r[0], int(r[1]), int(r[2]), float(r[3]), int(r[4]), float(r[5])) for r in rows]


@pytest.mark.parametrize("row", [r if r[3] == 1.0 else pytest.param(r, marks=pytest.mark.slow) for r in golden_l1_rows()],
                         ids=lambda r: f"{r[0]}{r[1]}-alpha{r[3]:g}")
def test_exact_coarse_solve_bounds_the_papers_multigrid_coarse(row):
    """Level 1: the paper's coarse solver is a V-cycle, the oracle's is exact
    (reading R9).  The dof counts match, and the exact coarse solve gives a
    condition estimate and an iteration count no larger than the printed
    ones (observed: 27-57% lower estimates at alpha >= 1)."""
    fam, p, dofs, alpha, its, cond = row
    top, A = build(fam, p, n=6, alpha=alpha)
    assert top.n_dofs == dofs
    H = HybridSchwarz(A, top, fam)
    b = np.random.default_rng(5).uniform(-1.0, 1.0, top.n_dofs)
    _, info = pcg(lambda v: A @ v, H.apply, b, rtol=1e-8, maxit=300, norm="preconditioned")
    assert info["iterations"] <= its
    assert lanczos_condest(info["alphas"], info["betas"]) <= 1.0 * cond


def test_vertex_stars_cover_and_reduce_to_the_default_for_h1():
    """Every dof lies in some star; the split stars omit exactly the cell
    interiors; for H(grad) the split stars are the default patches."""
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=4)
    for fam, p in (("CG", 4), ("Ned", 3), ("RT", 3)):
        top = Topology(X, C, element(3, fam, p))
        split, full = vertex_star_lists(top, False), vertex_star_lists(top, True)
        cover = np.zeros(top.n_dofs, dtype=bool)
        for a, b in zip(split, full):
            assert np.all(a < top.offset[3])
            extra = np.setdiff1d(b, a)
            assert np.all(extra >= top.offset[3]) and len(b) == len(a) + len(extra)
            cover[b] = True
        assert cover.all()
        if fam == "CG":
            assert all(np.array_equal(a, b) for a, b in zip(split, patch_lists(top, "CG")))


def test_comparator_lists_nest():
    """Type-I stars lie inside the every-kind (Hiptmair) stars, split stars
    inside full ones, and the full forms add only cell-interior dofs; the
    full potentials add the CG cell interiors as Ned type-II cell dofs."""
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=4)
    p = 4
    top = Topology(X, C, element(3, "Ned", p))
    forms = ("paper", "paper-full", "hiptmair", "hiptmair-full")
    L = {f: patch_lists(top, "Ned", f) for f in forms}
    for e in range(top.n_ent[1]):
        a, b, c, d = (set(L[f][e].tolist()) for f in forms)
        assert a <= b <= d and a <= c <= d
        assert all(i >= top.offset[3] for i in (b - a) | (d - c))
    cg_N = (1, p - 1, (p - 1) * (p - 2) // 2, (p - 1) * (p - 2) * (p - 3) // 6)
    split, full = potential_patches(top, cg_N), potential_patches(top, cg_N, full=True)
    for v, (Gs, Gf) in enumerate(zip(split, full)):
        n_cells = sum(1 for c in range(top.n_cells) if v in top.cells[c])
        assert Gf.shape[1] == Gs.shape[1] + n_cells * cg_N[3]
        assert abs(Gf[:, :Gs.shape[1]] - Gs).max() == 0
        assert np.all(Gf[:, Gs.shape[1]:].nonzero()[0] >= top.offset[3])


@pytest.mark.parametrize("p", [2, 3, pytest.param(4, marks=pytest.mark.slow)])
def test_curl_potentials_are_divergence_free(p):
    """The H(div) type-I potential columns are curls: div-div stiffness times
    every column vanishes (a wrong orientation sign or a non-curl column
    would not), and the Whitney column has unit fluxes on the (two or more)
    faces containing the edge."""
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=5)
    top = Topology(X, C, element(3, "RT", p))
    K = assemble(top, all_cell_matrices(top.el, top, alpha=1.0, beta=0.0))
    M = assemble(top, all_cell_matrices(top.el, top, alpha=0.0, beta=1.0))
    for full in (False, True):
        for G in curl_potential_patches(top, full):
            KG = (K @ G).toarray()
            assert abs(KG).max() <= 1e-11 * abs(K).max()
            assert (G.T @ M @ G).diagonal().min() > 0
            w = G[:, 0].toarray().ravel()
            w = w[w != 0]
            assert len(w) >= 2 and np.all(np.abs(w) == 1.0)


@pytest.mark.parametrize("fam,p,form", [("CG", 4, "paper"), ("Ned", 2, "paper"), ("RT", 2, "paper"),
                                         ("Ned", 3, "vertex"), ("RT", 3, "vertex-full"),
                                         ("Ned", 3, "hiptmair-full"), ("RT", 3, "paper-full"),
                                         ("RT", 3, "typeI"), ("RT", 3, "typeI-full")])
def test_sweep_symmetric_positive_and_product_of_propagators(fam, p, form):
    top, A = build(fam, p, n=1, jitter=0.0)
    H = HybridSchwarz(A, top, fam, decomposition=form)
    n = top.n_dofs
    Ad = A.toarray()
    I = np.eye(n)
    B = np.column_stack([H.apply(I[:, j]) for j in range(n)])
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    E = I
    for Bm, w in H.groups() + H.groups()[1::-1]:
        Bm_d = np.column_stack([Bm(I[:, j]) for j in range(n)])
        E = (I - Bm_d @ Ad / w) @ E
    assert np.abs((I - B @ Ad) - E).max() <= 1e-10


@pytest.mark.parametrize("fam,p", [("CG", 3), ("RT", 2), pytest.param("Ned", 2, marks=pytest.mark.slow)] +
                         [pytest.param(f, q, marks=pytest.mark.slow) for f, q in (("CG", 5), ("Ned", 3), ("RT", 3))])
def test_weights_interlace_exact_spectrum(fam, p):
    top, A = build(fam, p, n=2, jitter=0.1)
    H = HybridSchwarz(A, top, fam)
    for idx, solve, seed in ((H.add.I, H.B_interior, SEED_INTERIOR), (H.Gamma, H.B_interface, SEED_INTERFACE)):
        if len(idx) == 0:
            continue
        lo, hi = subspace_extremes(A, idx, solve, seed)
        Am = A[idx][:, idx].toarray()
        n = A.shape[0]
        cols = []
        for j in range(len(idx)):
            f = np.zeros(n)
            f[idx] = Am[:, j]
            cols.append(solve(f)[idx])
        ev = np.sort(np.linalg.eigvals(np.column_stack(cols)).real)
        assert ev[0] * (1 - 1e-9) <= lo <= hi <= ev[-1] * (1 + 1e-9)
        assert hi >= 0.95 * ev[-1]
