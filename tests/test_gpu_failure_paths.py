"""GPU checks of the solver's non-converged and degenerate paths, through the
C ABI.

* An iteration cap below the iterations needed: rz_solve returns
  RZ_ERR_NO_CONVERGENCE with the info filled -- exactly max_iter iterations,
  the recursive residual above rtol -- and the iterate is the oracle's PCG
  iterate after the same number of steps (same recursion in FP64, so within
  1e-10 relative), with and without captured iteration graphs.
* A zero column among several right-hand sides: it stops before the first
  iteration with x = 0, and the other columns still meet their tolerance.
* An uneven batch with one capped member: the batch returns
  RZ_ERR_NO_CONVERGENCE, that member's info says so, and the others still
  converge to the oracle's solutions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble
from oracle.pcg import pcg
from oracle.precond import HybridSchwarz
from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu

RZ_ERR_NO_CONVERGENCE = -6


def oracle_case(fam, p, n, seed):
    X, C = kuhn_mesh(n, 3, jitter=0.1, seed=seed)
    top = Topology(X, C, element(3, fam, p))
    A = assemble(top, all_cell_matrices(top.el, top))
    return X, C, top, A, HybridSchwarz(A, top, fam)


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("fam,p", [("CG", 4), ("Ned", 3)])
def test_iteration_cap_reports_no_convergence(fam, p, graphs):
    from paper_2506_17406_amd import rz
    X, C, top, A, H = oracle_case(fam, p, 2, 21)
    cap = 3
    prob = rz.Problem(X, C, p, fam, max_iter=cap, graphs=graphs)
    b = load_vectors(top.n_dofs, 22)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12, check=False)
    torch.cuda.synchronize()
    assert info["code"] == RZ_ERR_NO_CONVERGENCE and info["status"] == RZ_ERR_NO_CONVERGENCE
    assert info["iterations"] == cap
    assert info["rel_residual"] > 1e-12
    xo, io = pcg(lambda v: A @ v, H.apply, b, rtol=1e-12, maxit=cap)
    assert io["iterations"] == cap and not io["converged"]
    assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(info["rel_residual"] / io["rel_residual"] - 1.0) <= 1e-8
    with pytest.raises(rz.RzError):
        prob.solve(bt, torch.zeros_like(bt), rtol=1e-12)


def test_zero_column_stops_at_once():
    from paper_2506_17406_amd import rz
    X, C, top, A, H = oracle_case("RT", 3, 2, 23)
    prob = rz.Problem(X, C, 3, "RT")
    B = load_vectors(top.n_dofs, 24, n_rhs=3)
    B[:, 1] = 0.0
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().T
    Xt = torch.zeros_like(Bt)
    infos = prob.solve(Bt, Xt, rtol=1e-10)
    X_ = Xt.cpu().numpy()
    assert infos[1]["status"] == 0 and infos[1]["iterations"] == 0
    assert not np.any(X_[:, 1])
    for j in (0, 2):
        assert infos[j]["status"] == 0
        assert np.linalg.norm(B[:, j] - A @ X_[:, j]) <= 1.2e-10 * np.linalg.norm(B[:, j])


def test_batch_with_a_capped_member():
    from paper_2506_17406_amd import rz
    cases = [("CG", 3, 2, 25, 1000), ("Ned", 3, 2, 26, 4), ("RT", 3, 2, 27, 1000)]
    built = [oracle_case(fam, p, n, seed) + (cap, fam, p) for fam, p, n, seed, cap in cases]
    probs = [rz.Problem(X, C, p, fam, max_iter=cap) for X, C, top, A, H, cap, fam, p in built]
    batch = rz.Batch(probs)
    bs = [torch.from_numpy(load_vectors(c[2].n_dofs, 28 + i)[:, 0]).cuda() for i, c in enumerate(built)]
    xs = [torch.zeros_like(b) for b in bs]
    infos = batch.solve(bs, xs, rtol=1e-12, check=False)
    torch.cuda.synchronize()
    assert infos[0]["code"] == RZ_ERR_NO_CONVERGENCE
    assert infos[1]["status"] == RZ_ERR_NO_CONVERGENCE and infos[1]["iterations"] == 4
    for i in (0, 2):
        X, C, top, A, H, cap, fam, p = built[i]
        b = bs[i].cpu().numpy()
        xo, _ = pcg(lambda v: A @ v, H.apply, b, rtol=1e-12)
        assert infos[i]["status"] == 0
        assert np.linalg.norm(xs[i].cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    X, C, top, A, H, cap, fam, p = built[1]
    xo, _ = pcg(lambda v: A @ v, H.apply, bs[1].cpu().numpy(), rtol=1e-12, maxit=4)
    assert np.linalg.norm(xs[1].cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
