"""GPU parity of the multigrid V-cycle on W^k (rz_options.coarse =
RZ_COARSE_MG) against the oracle's (oracle.multigrid), through the C ABI,
on tetrahedra and triangles.

The hierarchy is the Kuhn meshes with n, n/2, ..., 1 cells per edge; the
problem's mesh is the jittered finest one (the prolongations use the
unperturbed positions, as the oracle's).  Bars: the hybrid weights
(including the V-cycle's rho_W) 1e-10 relative; apply_P max(1e-10, 10 u
kappa_pc) max |z| (explicit inverses on both sides here: the level
operators are inverted only on the coarsest mesh and in the edge stars);
solve: iteration counts within one, ||x - x_oracle|| <= 1e-10 ||x_oracle||
at rtol 1e-12, true residual 1e-10.  Multi-column and reduced-precision
handles use the same cycle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble
from oracle.pcg import pcg
from oracle.precond import AdditiveSchwarz, HybridSchwarz
from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu

CASES = [("CG", 3, 4), ("Ned", 3, 4), ("RT", 2, 4), ("Ned", 2, 8), ("CG", 2, 2), ("RT", 3, 2),
         # triangles (2D RT_p takes the H(curl) prolongation and smoother)
         ("CG", 4, 16, 2), ("Ned", 3, 16, 2), ("RT", 3, 16, 2), ("Ned", 5, 8, 2)]
_cache = {}


def hierarchy(n, d=3):
    out, m = [], n
    while True:
        out.append(kuhn_mesh(m, d))
        if m % 2 or m == 1:
            return out
        m //= 2


def setup(fam, p, n, d=3, pc="hybrid", precision="fp64"):
    key = (fam, p, n, d, pc, precision)
    if key not in _cache:
        from paper_2506_17406_amd import rz
        print(f"setup {key}", flush=True)
        X, C = kuhn_mesh(n, d, jitter=0.1, seed=81)
        okey = (fam, p, n, d)
        if okey not in _cache:
            top = Topology(X, C, element(d, fam, p))
            A = assemble(top, all_cell_matrices(top.el, top))
            _cache[okey] = (top, A, AdditiveSchwarz(A, top, fam, coarse_mg=n), {})
        top, A, Pa, pcs = _cache[okey]
        if pc not in pcs:
            pcs[pc] = Pa if pc == "additive" else HybridSchwarz(A, top, fam, additive=Pa)
        prob = rz.Problem(X, C, p, fam, pc=pc, precision=precision, coarse="mg", mg_meshes=hierarchy(n, d))
        _cache[key] = (top, A, pcs[pc], prob)
    return _cache[key]


def ids(c):
    return "{}{}-n{}".format(*c[:3]) + ("-2d" if len(c) > 3 and c[3] == 2 else "")


@pytest.mark.parametrize("pc", ["additive", "hybrid"])
@pytest.mark.parametrize("case", CASES, ids=ids)
def test_vcycle_apply_P_and_solve(case, pc):
    top, A, P, prob = setup(*case, pc=pc)
    if pc == "hybrid":
        rho = prob.pc_weights()
        assert abs(rho[0] / P.rho_I - 1) <= 1e-10 and abs(rho[1] / P.rho_Gamma - 1) <= 1e-10
        assert abs(rho[2] / P.rho_W - 1) <= 1e-10 and P.rho_W != 1.0
    r = load_vectors(top.n_dofs, 82)[:, 0]
    zt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt)
    torch.cuda.synchronize()
    ref = P.apply(r)
    assert np.abs(zt.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    b = load_vectors(top.n_dofs, 83)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    xo, io = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[8]], ids=ids)
def test_vcycle_multi_column(case):
    top, A, P, prob = setup(*case)
    B = load_vectors(top.n_dofs, 84, n_rhs=3)
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().T
    Zt, Xt = torch.zeros_like(Bt), torch.zeros_like(Bt)
    prob.apply_P(Bt, Zt)
    infos = prob.solve(Bt, Xt, rtol=1e-12)
    torch.cuda.synchronize()
    Z, X = Zt.cpu().numpy(), Xt.cpu().numpy()
    for j in range(3):
        ref = P.apply(B[:, j])
        assert np.abs(Z[:, j] - ref).max() <= 1e-10 * np.abs(ref).max()
        xo, io = pcg(lambda v: A @ v, P.apply, B[:, j], rtol=1e-12)
        assert abs(infos[j]["iterations"] - io["iterations"]) <= 1
        assert np.linalg.norm(X[:, j] - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", ["fp32-ir", "bf16-pc"])
def test_vcycle_reduced_precision(precision):
    top, A, P, prob = setup("Ned", 3, 4, precision=precision)
    b = load_vectors(top.n_dofs, 85)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    xo, io = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


def test_vcycle_errors():
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(4, 3, jitter=0.1, seed=81)
    with pytest.raises(rz.RzError) as e:           # the hierarchy does not start at the problem's mesh
        rz.Problem(X, C, 2, "CG", coarse="mg", mg_meshes=hierarchy(2))
    assert e.value.code == -3
    flags = np.zeros((len(C), 4), dtype=np.uint8)
    flags[0, 0] = 1
    with pytest.raises(rz.RzError) as e:           # Dirichlet + multigrid
        rz.Problem(X, C, 2, "CG", coarse="mg", mg_meshes=hierarchy(4), dirichlet_facet=flags)
    assert e.value.code in (-2, -3)
    for fam in ("NedTwo", "BDM"):                  # the hierarchy is built for the first-kind spaces
        with pytest.raises(rz.RzError) as e:
            rz.Problem(X, C, 2, fam, coarse="mg", mg_meshes=hierarchy(4))
        assert e.value.code == -2
