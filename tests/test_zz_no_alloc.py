"""rz_apply_A_noalloc (the operator apply for callers that cannot allocate
device memory) against rz_apply_A through the C ABI: two calls in a row on
one GPU, the second with a smaller input (another handle, fewer cells and
one column), must give rz_apply_A's results bit for bit (the same kernels in
the same order; only the cell-local work vectors live elsewhere), and both
must meet the oracle within 1e-12 max |y|.  A request beyond the static
array is refused with RZ_ERR_ARG."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import all_cell_matrices, assemble
from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu


def _case(fam, p, n, seed):
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(n, 3, jitter=0.1, seed=seed)
    top = Topology(X, C, element(3, fam, p))
    A = assemble(top, all_cell_matrices(top.el, top))
    return top, A, rz.Problem(X, C, p, fam, pc="additive")


def _cols(x):
    return torch.from_numpy(np.ascontiguousarray(x.T)).cuda().T


def test_noalloc_matches_apply_A_on_consecutive_calls():
    big = _case("Ned", 4, 3, 61)
    small = _case("CG", 3, 2, 62)
    for (top, A, prob), nr in ((big, 3), (small, 1)):
        x = load_vectors(top.n_dofs, 63, n_rhs=nr)
        xt = _cols(x)
        y_ref = torch.full_like(xt, np.nan)
        y_na = torch.full_like(xt, np.nan)
        prob.apply_A(xt, y_ref)
        prob.apply_A_noalloc(xt, y_na)
        torch.cuda.synchronize()
        a, b = y_ref.cpu().numpy(), y_na.cpu().numpy()
        assert np.array_equal(a, b)
        ref = A @ x
        assert np.abs(b - ref).max() <= 1e-12 * np.abs(ref).max()


def test_noalloc_refuses_requests_beyond_the_static_array():
    from paper_2506_17406_amd import rz
    top, A, prob = _case("Ned", 4, 3, 61)
    nr = 400                      # (84 + 96) * 256 * 8 bytes per column: 147 MB in all
    xt = torch.zeros(top.n_dofs, nr, dtype=torch.float64, device="cuda").T.contiguous().T
    yt = torch.zeros_like(xt)
    with pytest.raises(rz.RzError) as e:
        prob.apply_A_noalloc(xt, yt)
    assert e.value.code == -1 and "static" in str(e.value)
