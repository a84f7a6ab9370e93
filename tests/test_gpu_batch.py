"""GPU checks of the uneven batch (rz_batch_create / rz_batch_solve): problems
of different spaces, degrees, meshes, preconditioner forms and precisions
solved together, with their iteration chunks replayed from captured HIP
graphs.

Bars: every batch solution meets the oracle's (FP64 PCG to 1e-12 with the
same preconditioner form) within 1e-10 relative and takes the iteration
count of the same problem's own rz_solve within one.  The graphs are
replayed several times with eager work in between (separate solves, a
workspace reallocation that must force a re-capture, new solution vectors)
and every replay is checked.
"""
import time

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

# (dim, space, degree, cells per edge, preconditioner form, precision)
MEMBERS = [(3, "CG", 2, 3, "hybrid", "fp64"), (3, "Ned", 4, 2, "hybrid", "fp64"), (3, "CG", 6, 2, "hybrid", "fp32-pc"),
           (3, "RT", 3, 2, "additive", "fp64"), (2, "CG", 4, 4, "hybrid", "fp64"), (3, "Ned", 2, 1, "hybrid", "fp32-ir"),
           (3, "RT", 5, 1, "hybrid", "fp64"), (3, "Ned", 3, 2, "hybrid", "bf16-pc")]

_state = {}


def members():
    if "m" not in _state:
        from paper_2506_17406_amd import rz
        out = []
        for i, (d, fam, p, n, pc, prec) in enumerate(MEMBERS):
            X, C = kuhn_mesh(n, d, jitter=0.1 if d == 3 else 0.0, seed=40 + i)
            top = Topology(X, C, element(d, fam, p))
            A = assemble(top, all_cell_matrices(top.el, top))
            Pa = AdditiveSchwarz(A, top, fam)
            P = Pa if pc == "additive" else HybridSchwarz(A, top, fam, additive=Pa)
            prob = rz.Problem(X, C, p, fam, pc=pc, precision=prec)
            out.append((top, A, P, prob))
        _state["m"] = out
        _state["batch"] = rz.Batch([m[3] for m in out])
    return _state["m"], _state["batch"]


def check(ms, xs, infos, seed, own_its):
    for (top, A, P, prob), x, info, its in zip(ms, xs, infos, own_its or [None] * len(ms)):
        b = load_vectors(top.n_dofs, seed)[:, 0]
        xo, _ = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
        xv = x.cpu().numpy()
        assert info["status"] == 0
        assert np.linalg.norm(xv - xo) <= 1e-10 * np.linalg.norm(xo)
        if its is not None:
            assert abs(info["iterations"] - its) <= 1


def rhs(ms, seed):
    return [torch.from_numpy(load_vectors(m[0].n_dofs, seed)[:, 0]).cuda() for m in ms]


def test_batch_matches_oracle_and_own_solves():
    ms, batch = members()
    bs = rhs(ms, 50)
    own = []
    for (top, A, P, prob), b in zip(ms, bs):
        x = torch.zeros_like(b)
        own.append(prob.solve(b, x, rtol=1e-12)["iterations"])
    xs = [torch.zeros_like(b) for b in bs]
    t0 = time.perf_counter()
    infos = batch.solve(bs, xs, rtol=1e-12)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    check(ms, xs, infos, 50, own)
    # each member reports its own completion time and its handle's setup time
    assert all(0 < i["solve_ms"] <= wall_ms for i in infos)
    assert len({round(i["solve_ms"], 6) for i in infos}) > 1
    assert all(i["setup_ms"] > 0 for i in infos)
    # the refinement member ran its correction solves inside the batch
    ir = [i for (d, f, p, n, pc, prec), i in zip(MEMBERS, infos) if prec == "fp32-ir"]
    assert ir and all(i["outer_iterations"] >= 2 for i in ir)
    _state["xs"], _state["own"] = xs, own


def test_batch_graph_replays_with_eager_work_between():
    ms, batch = members()
    xs = _state.get("xs") or [torch.zeros(m[0].n_dofs, dtype=torch.float64, device="cuda") for m in ms]
    for k, seed in enumerate((51, 52, 53)):
        bs = rhs(ms, seed)
        for x in xs:
            x.zero_()
        infos = batch.solve(bs, xs, rtol=1e-12)
        torch.cuda.synchronize()
        check(ms, xs, infos, seed, None)
        # eager work between replays: a separate single solve on one member
        top, A, P, prob = ms[k % len(ms)]
        y = torch.zeros_like(bs[k % len(ms)])
        prob.solve(bs[k % len(ms)], y, rtol=1e-10)


def test_batch_recaptures_after_workspace_growth_and_new_vectors():
    ms, batch = members()
    # three columns on one member grow (reallocate) its Krylov workspace
    top, A, P, prob = ms[1]
    B3 = torch.from_numpy(np.ascontiguousarray(load_vectors(top.n_dofs, 54, n_rhs=3).T)).cuda().T
    X3 = torch.zeros_like(B3)
    prob.solve(B3, X3, rtol=1e-10)
    bs = rhs(ms, 55)
    xs = [torch.zeros_like(b) for b in bs]          # new solution vectors
    infos = batch.solve(bs, xs, rtol=1e-12)
    torch.cuda.synchronize()
    check(ms, xs, infos, 55, None)
