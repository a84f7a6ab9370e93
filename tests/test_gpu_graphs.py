"""rz_solve with captured iteration graphs (the default) against the same
solves launched kernel by kernel (eager handles), replayed several times
with eager work and synchronisations in between, every replay checked:
iteration counts equal and solutions within 1e-12 relative (the two runs
differ only in the order of FP64 atomic additions in the preconditioner).
Also: a workspace reallocation between replays (more columns) and a new
solution vector force a re-capture; the multi-column and mixed-precision
paths replay too.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu

CASES = [(3, "Ned", 4, 2, "hybrid", "fp64"), (3, "CG", 5, 2, "additive", "fp64"), (3, "RT", 3, 2, "hybrid", "fp32-pc"),
         (3, "Ned", 3, 2, "hybrid", "fp32-ir"), (2, "CG", 4, 4, "hybrid", "fp64"), (3, "CG", 4, 2, "hybrid", "bf16-pc")]


def pair(d, fam, p, n, pc, prec):
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(n, d, jitter=0.1 if d == 3 else 0.0, seed=60)
    g = rz.Problem(X, C, p, fam, pc=pc, precision=prec)
    e = rz.Problem(X, C, p, fam, pc=pc, precision=prec, graphs=False)
    return g, e


@pytest.mark.parametrize("case", CASES, ids=lambda c: "{}d-{}{}-n{}-{}-{}".format(*c))
def test_graph_replays_match_eager(case):
    g, e = pair(*case)
    x = torch.zeros(g.n_dofs, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for k in range(5):
        b = torch.from_numpy(load_vectors(g.n_dofs, 70 + k)[:, 0]).cuda()
        x.zero_()
        ig = g.solve(b, x, rtol=1e-11)
        xg = x.clone()
        xe = torch.zeros_like(x)
        ie = e.solve(b, xe, rtol=1e-11)
        torch.cuda.synchronize()
        assert abs(ig["iterations"] - ie["iterations"]) <= 1
        assert float((xg - xe).norm()) <= 1e-12 * float(xe.norm()) * max(1, ig["iterations"])
        # eager work between replays on the graph handle
        g.apply_A(xg, y)
        g.apply_P(b, y)
        if k == 2:
            # more columns: the workspace is reallocated, stale graphs must not run
            B = torch.from_numpy(np.ascontiguousarray(load_vectors(g.n_dofs, 80, n_rhs=3).T)).cuda().T
            X3 = torch.zeros_like(B)
            g.solve(B, X3, rtol=1e-10)
        if k == 3:
            x = torch.zeros_like(x)  # a new solution vector
