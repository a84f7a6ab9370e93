"""Oracle pins at the mesh / solver level (no GPU).

* global dof counts printed in the paper's tables (tests/golden);
* Kuhn entity counts and star sizes (Sec. 6.1: 14 edges, 36 faces, 24 cells);
* maximum patch sizes printed in the paper (tests/golden);
* global identities: mass of gradients = H(grad) stiffness, curl grad = 0,
  exactness ranks on a one-cube mesh;
* PCG against a dense direct solve on tiny meshes; symmetry and positivity
  of the preconditioner; bounded condition estimates;
* optimal energy-norm convergence O(h^p) on manufactured solutions.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble, element_apply, functional_load
from oracle.pcg import lanczos_condest, pcg
from oracle.precond import AdditiveSchwarz, patch_lists, potential_patches, vertex_star_lists
from paper_2506_17406_amd.workloads import kuhn_counts, kuhn_mesh, load_vectors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


def per_entity(space, p):
    """dofs per (vertex, edge, face, cell) from the type-I/II counts."""
    if space == "CG":
        return (1, p - 1, (p - 1) * (p - 2) // 2, (p - 1) * (p - 2) * (p - 3) // 6)
    if space == "Ned":
        return (0, p, (p - 1) * (p + 2) // 2 + (p - 1) * (p - 2) // 2,
                (p - 1) * (p - 2) * (2 * p + 3) // 6 + (p - 1) * (p - 2) * (p - 3) // 6)
    return (0, 0, 1 + (p - 1) * (p + 2) // 2,
            (p - 1) * (p * p + 4 * p + 6) // 6 + (p - 1) * (p - 2) * (2 * p + 3) // 6)


@pytest.mark.parametrize("space", ["CG", "Ned", "RT"])
@pytest.mark.parametrize("p", [2, 3] + [pytest.param(q, marks=pytest.mark.slow) for q in (5, 7)])
def test_per_entity_counts_match_elements(space, p):
    assert tuple(element(3, space, p).counts()) == per_entity(space, p)


def test_paper_dof_counts():
    for space, level, n, p, dofs in _read("paper_dof_counts.txt"):
        n, p, dofs = int(n), int(p), int(dofs)
        total = sum(a * b for a, b in zip(kuhn_counts(n), per_entity(space, p)))
        assert total == dofs, (space, level, p)


@pytest.mark.parametrize("space,p", [("CG", 3), ("Ned", 3), ("RT", 3), ("CG", 5)])
def test_topology_dof_count_level0(space, p):
    X, C = kuhn_mesh(3)
    top = Topology(X, C, element(3, space, p))
    expect = {int(r[4]) for r in _read("paper_dof_counts.txt") if r[0] == space and r[1] == "0" and int(r[3]) == p}
    assert {top.n_dofs} == expect
    assert tuple(top.n_ent) == kuhn_counts(3)
    # numbering contract: interiors last and contiguous, every dof used
    assert np.array_equal(np.unique(top.cell_dofs), np.arange(top.n_dofs))
    inner = element(3, space, p).interior()
    if inner.any():
        assert top.cell_dofs[:, inner].min() == top.offset[3]


def test_star_sizes():
    X, C = kuhn_mesh(4)
    top = Topology(X, C, element(3, "CG", 2))
    edges_of, faces_of = top.vertex_star()
    v = 2 + 5 * (2 + 5 * 2)   # an interior vertex
    assert len(edges_of[v]) == 14 and len(faces_of[v]) == 36
    assert np.sum(np.any(top.cells == v, axis=1)) == 24
    assert max(len(f) for f in top.edge_faces()) == 6


def test_paper_patch_sizes_p4():
    X, C = kuhn_mesh(3)
    golden = {(r[0], r[1], int(r[2])): int(r[3]) for r in _read("paper_patch_sizes.txt")}
    cg = Topology(X, C, element(3, "CG", 4))
    assert max(len(i) for i in patch_lists(cg, "CG")) == golden[("CG", "vertex_star_interface", 4)]
    ned = Topology(X, C, element(3, "Ned", 4))
    assert max(len(i) for i in patch_lists(ned, "Ned")) == golden[("Ned", "edge_star_typeI_interface", 4)]
    assert max(G.shape[1] for G in potential_patches(ned, (1, 3, 3))) == golden[("Ned", "vertex_potential_interface", 4)]
    rt = Topology(X, C, element(3, "RT", 4))
    assert max(len(i) for i in patch_lists(rt, "RT")) == golden[("RT", "edge_star_interface", 4)]
    assert max(len(i) for i in vertex_star_lists(cg, True)) == golden[("CG", "vertex_star_full", 4)]
    assert max(len(i) for i in vertex_star_lists(cg, False)) == golden[("CG", "vertex_star_interface", 4)]


def test_paper_patch_sizes_p10_closed_form():
    # interior vertex star: 14 edges, 36 faces; interior edge: 6 faces
    golden = {(r[0], r[1], int(r[2])): int(r[3]) for r in _read("paper_patch_sizes.txt")}
    for p in (4, 10):
        cg = per_entity("CG", p)
        assert 1 + 14 * cg[1] + 36 * cg[2] == golden[("CG", "vertex_star_interface", p)]
        assert 1 + 14 * cg[1] + 36 * cg[2] + 24 * cg[3] == golden[("CG", "vertex_star_full", p)]
        assert 1 + 6 * (p - 1) * (p + 2) // 2 == golden[("Ned", "edge_star_typeI_interface", p)]
        assert 6 * per_entity("RT", p)[2] == golden[("RT", "edge_star_interface", p)]


def _global_gradient(top_ned, top_cg, p):
    """Sparse n_Ned x n_CG discrete gradient: Whitney incidence plus the
    identity CG type-I -> Ned type-II (eq:d-preserves-basis-functions-global)."""
    rows, cols, vals = [], [], []
    for e, (a, b) in enumerate(top_ned.ent_tuples[1]):
        w = top_ned.entity_dofs(1, e, kinds=("W",))[0]
        rows += [w, w]; cols += [top_cg.offset[0] + a, top_cg.offset[0] + b]; vals += [-1.0, 1.0]
    for l in (1, 2, 3):
        for ent in range(top_ned.n_ent[l]):
            ii = top_ned.entity_dofs(l, ent, kinds=("II",))
            cc = top_cg.entity_dofs(l, ent)
            assert len(ii) == len(cc)
            rows += ii; cols += cc; vals += [1.0] * len(ii)
    return sp.csr_matrix((vals, (rows, cols)), shape=(top_ned.n_dofs, top_cg.n_dofs))


@pytest.mark.parametrize("p", [2, 3])
def test_global_gradient_identities(p):
    X, C = kuhn_mesh(2, jitter=0.1, seed=3)
    cg, ned = Topology(X, C, element(3, "CG", p)), Topology(X, C, element(3, "Ned", p))
    G = _global_gradient(ned, cg, p)
    K_cg = assemble(cg, all_cell_matrices(cg.el, cg, alpha=1.0, beta=0.0))
    M_ned = assemble(ned, all_cell_matrices(ned.el, ned, alpha=0.0, beta=1.0))
    K_ned = assemble(ned, all_cell_matrices(ned.el, ned, alpha=1.0, beta=0.0))
    assert abs(G.T @ M_ned @ G - K_cg).max() < 1e-11 * abs(K_cg).max()
    assert abs(K_ned @ G).max() < 1e-11 * abs(K_ned).max()


def test_exactness_ranks_one_cube():
    X, C = kuhn_mesh(1)
    p = 2
    tops = {s: Topology(X, C, element(3, s, p)) for s in ("CG", "Ned", "RT")}
    kern = {}
    for s, t in tops.items():
        K = assemble(t, all_cell_matrices(t.el, t, alpha=1.0, beta=0.0)).toarray()
        ev = np.linalg.eigvalsh(K)
        kern[s] = int(np.sum(ev < 1e-10 * ev.max()))
    n = {s: t.n_dofs for s, t in tops.items()}
    assert kern["CG"] == 1                                 # constants
    assert kern["Ned"] == n["CG"] - 1                      # ker curl = grad CG
    assert kern["RT"] == n["Ned"] - kern["Ned"]            # ker div = curl Ned
    # div onto DG_{p-1} (dim per cell p(p+1)(p+2)/6): RT dofs - ker div
    assert n["RT"] - kern["RT"] == 6 * p * (p + 1) * (p + 2) // 6


def _setup(d, space, p, n, jitter=0.1, seed=2):
    X, C = kuhn_mesh(n, d, jitter=jitter, seed=seed)
    top = Topology(X, C, element(d, space, p))
    Ac = all_cell_matrices(top.el, top)
    A = assemble(top, Ac)
    return top, Ac, A


@pytest.mark.parametrize("d,space,p,n", [(2, "CG", 4, 4), (3, "CG", 3, 2), (3, "Ned", 2, 2),
                                         (3, "Ned", 3, 1), (3, "RT", 3, 2), (3, "RT", 2, 1)])
def test_pcg_matches_dense_solve(d, space, p, n):
    top, Ac, A = _setup(d, space, p, n, jitter=0.0 if d == 2 else 0.1)
    P = AdditiveSchwarz(A, top, space)
    b = load_vectors(top.n_dofs, 1)[:, 0]
    Ad = A.toarray()
    xs = np.linalg.solve(Ad, b)
    x, info = pcg(lambda v: A @ v, P.apply, b, rtol=1e-14, maxit=500)
    assert info["converged"]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-11
    # the matrix-free element apply agrees with the assembled operator
    assert np.abs(element_apply(top, Ac, b) - A @ b).max() < 1e-12 * np.abs(A @ b).max()


@pytest.mark.parametrize("d,space,p,n", [(2, "CG", 4, 4), (3, "CG", 3, 2), (3, "Ned", 3, 1), (3, "RT", 2, 2)])
def test_preconditioner_symmetric_positive(d, space, p, n):
    top, Ac, A = _setup(d, space, p, n)
    P = AdditiveSchwarz(A, top, space)
    Pm = np.stack([P.apply(e) for e in np.eye(top.n_dofs)], axis=1)
    assert np.abs(Pm - Pm.T).max() < 1e-12 * np.abs(Pm).max()
    assert np.linalg.eigvalsh(0.5 * (Pm + Pm.T)).min() > 0


@pytest.mark.slow
@pytest.mark.parametrize("space", ["CG", "Ned", "RT"])
def test_condest_bounded_in_p(space):
    """p-robustness (Sec. 6, thm:generic-subspace-decomp-interface-interior-split):
    the preconditioned condition number stays bounded as p grows."""
    conds = []
    for p in (2, 3, 4):
        top, Ac, A = _setup(3, space, p, 2, jitter=0.0)
        P = AdditiveSchwarz(A, top, space)
        b = load_vectors(top.n_dofs, 1)[:, 0]
        _, info = pcg(lambda v: A @ v, P.apply, b, rtol=1e-10)
        conds.append(lanczos_condest(info["alphas"], info["betas"]))
    assert max(conds) < 25.0
    assert conds[-1] < 2.0 * conds[0]


def _fields(space):
    pi = np.pi
    if space == "CG":
        u = lambda x: (np.sin(pi * x[:, 0]) * np.cos(pi * x[:, 1]) * np.exp(x[:, 2]))[:, None]
        du = lambda x: np.stack([pi * np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1]) * np.exp(x[:, 2]),
                                 -pi * np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]) * np.exp(x[:, 2]),
                                 np.sin(pi * x[:, 0]) * np.cos(pi * x[:, 1]) * np.exp(x[:, 2])], axis=1)
        return u, du
    if space == "Ned":
        # u = (sin y, sin z, sin x): curl u = (-cos z, -cos x, -cos y)
        u = lambda x: np.stack([np.sin(x[:, 1]), np.sin(x[:, 2]), np.sin(x[:, 0])], axis=1) * 3
        du = lambda x: -np.stack([np.cos(x[:, 2]), np.cos(x[:, 0]), np.cos(x[:, 1])], axis=1) * 3
        return u, du
    # u = (sin(2x) y, cos z x, exp(y)): div u = 2 cos(2x) y
    u = lambda x: np.stack([np.sin(2 * x[:, 0]) * x[:, 1], np.cos(x[:, 2]) * x[:, 0], np.exp(x[:, 1])], axis=1)
    du = lambda x: (2 * np.cos(2 * x[:, 0]) * x[:, 1])[:, None]
    return u, du


@pytest.mark.slow
@pytest.mark.parametrize("space,p", [(s, p) for s in ("CG", "Ned", "RT") for p in (1, 2, 3, 4)])
def test_manufactured_energy_convergence(space, p):
    """The Galerkin solution is the a-projection of u*, so its energy error
    a(u* - u_h, u* - u_h) = a(u*, u*) - b^T x decays like h^{2p}.  At p = 3, 4
    the cell type-I bubbles of Ned and RT take part (observed rates on
    n = 2 -> 4: CG 2.82 / 3.78, Ned 2.89 / 3.91, RT 2.92 / 3.95)."""
    u, du = _fields(space)
    errs = []
    for n in (2, 4):
        top, Ac, A = _setup(3, space, p, n, jitter=0.1, seed=5)
        b, energy = functional_load(top.el, top, u, du)
        x = sp.linalg.spsolve(A.tocsc(), b)
        errs.append(np.sqrt(max(energy - b @ x, 0.0)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p - 0.35, (errs, rate)
