"""GPU parity of the Dirichlet boundary (rz_options.dirichlet_facet; the
problem on X^k_{p,D}, Sec. 5) against the oracle, through the C ABI.

* the removed dofs equal the oracle's (bit-exact), and so do the plain
  patch lists restricted to X^k_{p,D};
* apply_A = M A M x and apply_P = the oracle's restricted preconditioner
  applied to M r (M: zero on the removed dofs; the library ignores the
  removed entries of its inputs and writes zeros there): 1e-12 / 1e-10
  relative;
* solve (FP64 hybrid and additive, FP32 refinement, bfloat16
  preconditioner, and a batch with Dirichlet members): the oracle's PCG
  on M A M with M b, solutions within 1e-10 relative at rtol 1e-12, zero on
  the removed dofs, iteration counts within one (FP64) or two (reduced
  precision);
* a marked facet inside the mesh is RZ_ERR_MESH.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle.element import element
from oracle.mesh import Topology, dirichlet_dofs
from oracle.operator import all_cell_matrices, assemble
from oracle.pcg import pcg
from oracle.precond import AdditiveSchwarz, HybridSchwarz, patch_lists
from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu


def boundary_flags(C, X, where):
    d = C.shape[1] - 1
    flags = np.zeros((len(C), d + 1), dtype=np.uint8)
    for c in range(len(C)):
        for j in range(d + 1):
            f = X[np.delete(C[c], j)]
            on0 = np.all(np.isclose(f, 0.0), axis=0)
            on1 = np.all(np.isclose(f, 1.0), axis=0)
            if (where == "all" and np.any(on0 | on1)) or (where == "face" and on0[0]):
                flags[c, j] = 1
    return flags


CASES = [(2, "CG", 4, 4, "all"), (3, "CG", 3, 2, "face"), (3, "CG", 5, 2, "all"), (3, "Ned", 3, 2, "all"),
         (3, "Ned", 4, 2, "face"), (3, "RT", 3, 2, "face"), (3, "RT", 4, 2, "all"), (3, "Ned", 1, 2, "face"),
         (2, "Ned", 4, 4, "all"), (2, "RT", 3, 4, "face"), (3, "NedTwo", 2, 2, "face"), (3, "BDM", 2, 2, "all")]
_cache = {}


def setup(d, fam, p, n, where, pc="hybrid", precision="fp64"):
    key = (d, fam, p, n, where, pc, precision)
    if key not in _cache:
        from paper_2506_17406_amd import rz
        X, C = kuhn_mesh(n, d, jitter=0.1 if d == 3 else 0.0, seed=71)
        flags = boundary_flags(C, X, where)
        okey = key[:5]
        if okey not in _cache:
            top = Topology(X, C, element(d, fam, p))
            A = assemble(top, all_cell_matrices(top.el, top))
            D = dirichlet_dofs(top, C, flags)
            keep = np.ones(top.n_dofs)
            keep[D] = 0.0
            M = sp.diags(keep)
            Pa = AdditiveSchwarz(A, top, fam, dirichlet=D)
            _cache[okey] = (top, A, (M @ A @ M).tocsr(), keep.astype(bool), D, Pa, {})
        top, A, Ad, keep, D, Pa, pcs = _cache[okey]
        if pc not in pcs:
            pcs[pc] = Pa if pc == "additive" else HybridSchwarz(A, top, fam, additive=Pa)
        prob = rz.Problem(X, C, p, fam, pc=pc, precision=precision, dirichlet_facet=flags)
        _cache[key] = (top, A, Ad, keep, D, pcs[pc], prob)
    return _cache[key]


def ids(c):
    return "{}d-{}{}-n{}-{}".format(*c)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_removed_dofs_and_restricted_patches(case):
    top, A, Ad, keep, D, P, prob = setup(*case)
    assert np.array_equal(prob.dirichlet_dofs(), D)
    cd, ptr, dofs = prob.export_topology()
    lists = [idx[keep[idx]] for idx in patch_lists(top, case[1])]
    lists = [idx for idx in lists if len(idx)]
    assert len(ptr) - 1 == len(lists)
    for k, idx in enumerate(lists):
        assert np.array_equal(dofs[ptr[k]:ptr[k + 1]], idx)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_apply_A_restricted(case):
    top, A, Ad, keep, D, P, prob = setup(*case)
    x = load_vectors(top.n_dofs, 72)[:, 0]          # arbitrary entries on the removed dofs too
    yt = torch.full((top.n_dofs,), np.nan, dtype=torch.float64, device="cuda")
    prob.apply_A(torch.from_numpy(x).cuda(), yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    ref = Ad @ x
    assert np.all(y[~keep] == 0.0)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("pc", ["additive", "hybrid"])
@pytest.mark.parametrize("case", CASES, ids=ids)
def test_apply_P_and_solve_restricted(case, pc):
    top, A, Ad, keep, D, P, prob = setup(*case, pc=pc)
    if pc == "hybrid":
        rho = prob.pc_weights()
        assert abs(rho[0] / P.rho_I - 1) <= 1e-10 and abs(rho[1] / P.rho_Gamma - 1) <= 1e-10
    r = load_vectors(top.n_dofs, 73)[:, 0]
    zt = torch.full((top.n_dofs,), np.nan, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    ref = P.apply(r * keep)
    assert np.all(z[~keep] == 0.0)
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    b = load_vectors(top.n_dofs, 74)[:, 0]
    bt = torch.from_numpy(b).cuda()
    # start from ones on the removed dofs (the solve must reset them) and zero elsewhere
    xt = torch.from_numpy((~keep).astype(np.float64)).cuda()
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    xo, io = pcg(lambda v: Ad @ v, P.apply, b * keep, rtol=1e-12)
    assert np.all(x[~keep] == 0.0)
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", ["fp32-ir", "bf16-pc"])
@pytest.mark.parametrize("case", [CASES[3], CASES[6]], ids=ids)
def test_reduced_precision_solves_restricted(case, precision):
    top, A, Ad, keep, D, P, prob = setup(*case, precision=precision)
    b = load_vectors(top.n_dofs, 75)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    xo, io = pcg(lambda v: Ad @ v, P.apply, b * keep, rtol=1e-12)
    assert np.all(x[~keep] == 0.0)
    assert np.linalg.norm(b * keep - Ad @ x) <= 1e-10 * np.linalg.norm(b * keep)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    if precision == "fp32-ir":
        assert info["outer_iterations"] >= 2
    else:
        assert abs(info["iterations"] - io["iterations"]) <= 2


def test_batch_with_dirichlet_members():
    from paper_2506_17406_amd import rz
    members = [setup(*CASES[1]), setup(*CASES[3], precision="fp32-ir"), setup(3, "Ned", 3, 2, "all", pc="additive")]
    batch = rz.Batch([m[-1] for m in members])
    bs = [torch.from_numpy(load_vectors(m[0].n_dofs, 76)[:, 0]).cuda() for m in members]
    xs = [torch.zeros_like(b) for b in bs]
    infos = batch.solve(bs, xs, rtol=1e-12)
    torch.cuda.synchronize()
    for (top, A, Ad, keep, D, P, prob), b, x, info in zip(members, bs, xs, infos):
        bn = b.cpu().numpy()
        xo, _ = pcg(lambda v: Ad @ v, P.apply, bn * keep, rtol=1e-12)
        xv = x.cpu().numpy()
        assert info["status"] == 0
        assert np.all(xv[~keep] == 0.0)
        assert np.linalg.norm(xv - xo) <= 1e-10 * np.linalg.norm(xo)
    batch.close()


def test_interior_facet_is_rejected():
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(2, 3)
    flags = np.zeros((len(C), 4), dtype=np.uint8)
    for j in range(4):
        f = set(np.delete(C[0], j).tolist())
        if sum(f <= set(c.tolist()) for c in C) == 2:
            flags[0, j] = 1
            break
    with pytest.raises(rz.RzError) as e:
        rz.Problem(X, C, 2, "CG", dirichlet_facet=flags)
    assert e.value.code == -3
