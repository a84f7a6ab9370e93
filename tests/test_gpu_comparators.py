"""GPU parity of the comparator decompositions of Sec. 6 against the
oracle, through the C ABI, in the additive and the symmetric multiplicative
hybrid form: PAFW(0)(X^k_Gamma) + J(X^k_I) ("vertex") and the full vertex
stars PAFW(0)(X^k) ("vertex-full") for every space; the default
decompositions without the split ("paper-full": H(curl) PH(X^0, X^{1,I}),
H(div) PAFW(1)(X^2)); the standard Hiptmair-Toselli decompositions of
H(curl) PH(X^0_Gamma, X^1_Gamma) + J ("hiptmair") and PH(X^0, X^1)
("hiptmair-full"); the type-I Hiptmair-Toselli decompositions
PH(X^{k-1,I}, X^{k,I}) with and without the split ("typeI", "typeI-full";
for H(div) built from curl potentials).  2D H(curl) and H(div) take the
H(curl) forms with the dimensions shifted (2D RT_p is the quarter turn of
2D Ned_p); the second-kind NedTwo_p and BDM_p those of H(curl) and H(div)
with potentials from CG_{p+1} and NedTwo_{p+1}.
The standard H(div) Hiptmair-Toselli decomposition (face stars and NedTwo
edge-star potentials with the regularising mass 1e-8 beta,
eq:local-potential-problem-added-mass) meets the same bars although its
potential matrices have condition numbers of 1e9-1e11 (see its test).

Sizes: meshes of 6-162 cells, degrees 2-8, seeded jitter and load vectors;
the largest full stars near the 2048-dof patch limit (H(grad) p = 8: 1695,
H(curl) p = 5: 1510, H(div) p = 5: 1980); degenerate cases: no interior dofs
(both forms coincide), a single cell, a mesh without interior vertices.
Bars, as for the default decompositions:
* group weights equal to the oracle's within 1e-10 (the full form's empty
  Jacobi group has weight 1);
* apply_P -- max |z_gpu - z_oracle| <= 1e-10 max |z_oracle|;
* solve   -- iteration counts within one, true residual under the oracle's A
             <= 1e-10, ||x_gpu - x_oracle|| <= 1e-10 ||x_oracle|| at rtol 1e-12.
A full star above 2048 dofs is refused with RZ_ERR_UNSUPPORTED at setup,
and so are decompositions not built for the space (before device work).
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

# (dim, space, degree, cells per edge (0 = a single tetrahedron), jitter)
CASES = [(3, "CG", 4, 2, 0.1), (3, "Ned", 3, 2, 0.1), (3, "Ned", 4, 2, 0.1), (3, "RT", 3, 2, 0.1),
         (3, "RT", 4, 3, 0.0), (2, "CG", 4, 3, 0.1),
         # no interior dofs, no interior vertex, a single cell
         (3, "Ned", 2, 2, 0.1), (3, "CG", 5, 1, 0.0), (3, "RT", 3, 0, 0.0),
         # the largest full stars below the patch limit
         (3, "CG", 8, 2, 0.1), (3, "Ned", 5, 2, 0.1), (3, "RT", 5, 2, 0.1)]
OTHER = [(3, "Ned", 3, 2, 0.1), (3, "Ned", 4, 2, 0.1), (3, "Ned", 2, 2, 0.1), (3, "Ned", 3, 0, 0.0),
         (3, "Ned", 6, 2, 0.1)]
SETS = ([(c, f) for f in ("vertex", "vertex-full") for c in CASES] +
        [(c, "paper-full") for c in [(3, "CG", 4, 2, 0.1), (2, "CG", 4, 3, 0.1), (3, "RT", 4, 2, 0.1),
                                     (3, "RT", 3, 0, 0.0), (3, "RT", 6, 2, 0.1)] + OTHER] +
        [(c, f) for f in ("hiptmair", "hiptmair-full") for c in OTHER] +
        [(c, f) for f in ("typeI", "typeI-full")
         for c in [(3, "RT", 3, 2, 0.1), (3, "RT", 4, 3, 0.0), (3, "RT", 2, 2, 0.1), (3, "RT", 3, 0, 0.0),
                   (3, "RT", 6, 2, 0.1), (3, "Ned", 3, 2, 0.1)]] +
        # 2D H(curl) and H(div) (the quarter turn): every decomposition
        [(c, f) for f in ("paper-full", "vertex", "vertex-full", "hiptmair", "hiptmair-full", "typeI")
         for c in [(2, "Ned", 4, 3, 0.1), (2, "RT", 5, 3, 0.1)]] +
        # the second-kind spaces
        [((3, "NedTwo", 3, 2, 0.1), f) for f in ("paper-full", "vertex", "vertex-full", "hiptmair",
                                                 "hiptmair-full", "typeI")] +
        [((3, "BDM", 3, 2, 0.1), f) for f in ("paper-full", "vertex", "vertex-full", "typeI", "typeI-full")])
PCS = ["additive", "hybrid"]
_cache = {}


def setup_case(d, fam, p, n, jit, form, pc):
    key = (d, fam, p, n, jit, form, pc)
    if key not in _cache:
        from paper_2506_17406_amd import rz
        if n == 0:
            X = np.array([[0.1, 0.0, 0.05], [1.0, 0.2, 0.0], [0.3, 0.9, 0.1], [0.2, 0.3, 1.1]])
            C = np.array([[2, 0, 3, 1]])
        else:
            X, C = kuhn_mesh(n, d, jitter=jit, seed=13)
        base = (d, fam, p, n, jit, form, "additive")
        if base in _cache:
            top, A, P_add = _cache[base][:3]
        else:
            top = Topology(X, C, element(d, fam, p))
            A = assemble(top, all_cell_matrices(top.el, top))
            P_add = AdditiveSchwarz(A, top, fam, decomposition=form)
        P = P_add if pc == "additive" else HybridSchwarz(A, top, fam, additive=P_add)
        print(f"setup {fam}{p} n={n} {form} {pc} dofs={top.n_dofs}", flush=True)
        prob = rz.Problem(X, C, p, fam, pc=pc, decomposition=form)
        assert prob.n_dofs == top.n_dofs
        _cache[key] = (top, A, P, prob)
    return _cache[key]


def ids(v):
    c, f = v
    return ("{}d-{}{}-n{}".format(*c[:4]) if c[3] else "{}d-{}{}-tet".format(*c[:3])) + "-" + f


@pytest.mark.parametrize("pc", PCS)
@pytest.mark.parametrize("cf", SETS, ids=ids)
def test_apply_P(cf, pc):
    case, form = cf
    top, A, P, prob = setup_case(*case, form, pc)
    if pc == "hybrid":
        rho = prob.pc_weights()
        assert abs(rho[0] / P.rho_I - 1) <= 1e-10 and abs(rho[1] / P.rho_Gamma - 1) <= 1e-10 and rho[2] == 1.0
        if form.endswith("full"):
            assert rho[0] == 1.0
    r = load_vectors(top.n_dofs, 16)[:, 0]
    zt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt)
    torch.cuda.synchronize()
    ref = P.apply(r)
    assert np.abs(zt.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("pc", PCS)
@pytest.mark.parametrize("cf", SETS, ids=ids)
def test_solve(cf, pc):
    case, form = cf
    top, A, P, prob = setup_case(*case, form, pc)
    b = load_vectors(top.n_dofs, 17)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    xo, io = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


def test_full_star_above_patch_limit_is_refused():
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(2, 3, jitter=0.1, seed=13)
    with pytest.raises(rz.RzError) as e:
        rz.Problem(X, C, 6, "Ned", decomposition="vertex-full")   # interior star: 2604 dofs
    assert e.value.code == -2 and "2048" in str(e.value)
    prob = rz.Problem(X, C, 6, "Ned", decomposition="vertex")      # split star: 1164 dofs
    assert prob.n_dofs > 0


MULTI = [((3, "RT", 5, 2, 0.1), "vertex-full"), ((3, "CG", 8, 2, 0.1), "vertex-full"),
         ((3, "Ned", 4, 2, 0.1), "hiptmair-full"), ((3, "RT", 3, 2, 0.1), "typeI"),
         ((3, "RT", 4, 3, 0.0), "typeI-full")]


@pytest.mark.parametrize("pc", PCS)
@pytest.mark.parametrize("cf", MULTI, ids=ids)
@pytest.mark.parametrize("nr", [3, 9])
def test_multi_rhs(cf, nr, pc):
    """Several right-hand sides at once: the large-patch kernel one column
    group at a time, the small potentials through the patch GEMM at >= 8
    columns; per-column results are the oracle's."""
    case, form = cf
    top, A, P, prob = setup_case(*case, form, pc)
    B = load_vectors(top.n_dofs, 27, n_rhs=nr)
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().T
    Zt = torch.zeros_like(Bt)
    prob.apply_P(Bt, Zt)
    Xt = torch.zeros_like(Bt)
    infos = prob.solve(Bt, Xt, rtol=1e-12)
    torch.cuda.synchronize()
    Z, X = Zt.cpu().numpy(), Xt.cpu().numpy()
    for j in range(nr):
        ref = P.apply(B[:, j])
        assert np.abs(Z[:, j] - ref).max() <= 1e-10 * np.abs(ref).max()
        xo, io = pcg(lambda v: A @ v, P.apply, B[:, j], rtol=1e-12)
        assert abs(infos[j]["iterations"] - io["iterations"]) <= 1
        assert np.linalg.norm(X[:, j] - xo) <= 1e-10 * np.linalg.norm(xo)


REDUCED = [((3, "RT", 5, 2, 0.1), "vertex-full"), ((3, "CG", 8, 2, 0.1), "vertex-full"),
           ((3, "Ned", 4, 2, 0.1), "hiptmair"), ((3, "RT", 4, 3, 0.0), "typeI-full")]


@pytest.mark.parametrize("prec", ["fp32-pc", "bf16-pc", "fp32-ir"])
@pytest.mark.parametrize("cf", REDUCED, ids=ids)
def test_reduced_precision(cf, prec):
    """The comparators under the reduced-precision modes (FP32 and bfloat16
    patch copies of up to 1980-dof patches, FP32 refinement): the
    preconditioner within the copies' rounding of the oracle's (1e-4 FP32,
    1e-2 bfloat16), and solves to the FP64 tolerance whose solution is the
    oracle's within 1e-10."""
    from paper_2506_17406_amd import rz
    case, form = cf
    top, A, P, _ = setup_case(*case, form, "hybrid")
    d, fam, p, n, jit = case
    X, C = kuhn_mesh(n, d, jitter=jit, seed=13)
    prob = rz.Problem(X, C, p, fam, precision=prec, decomposition=form)
    r = load_vectors(top.n_dofs, 37)[:, 0]
    zt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt, fp32=True)
    torch.cuda.synchronize()
    ref = P.apply(r)
    err = np.abs(zt.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= (1e-2 if prec == "bf16-pc" else 1e-4)
    b = load_vectors(top.n_dofs, 38)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    x = xt.cpu().numpy()
    assert info["status"] == 0
    xo, _ = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


# ---- the standard H(div) Hiptmair-Toselli decomposition --------------------
U64 = 2.0 ** -53
HDIV_HT = [(3, "RT", 2, 1, 0.1), (3, "RT", 3, 2, 0.1), (3, "BDM", 2, 1, 0.1)]


def _kappa_pc(P):
    """Largest 2-norm condition number of the matrices the additive form
    factors (patches, potentials, coarse): the NedTwo potentials carry the
    regularising mass 1e-8 beta (eq:local-potential-problem-added-mass), so
    theirs is about 1e8."""
    add = getattr(P, "add", P)
    ks = [np.linalg.cond(np.tril(F[0])) ** 2 for _, F in add.patches + add.potentials]
    ks.append(np.linalg.cond(np.tril(add.coarse[0])) ** 2)
    return max(ks)


@pytest.mark.parametrize("pc", PCS)
@pytest.mark.parametrize("form", ["hiptmair", "hiptmair-full"])
@pytest.mark.parametrize("case", HDIV_HT, ids=lambda c: "{}d-{}{}-n{}".format(*c[:4]))
def test_hdiv_hiptmair(case, form, pc):
    """PH(X^1_Gamma, X^2_Gamma) + J and PH(X^1, X^2) for H(div)
    (eq:pavarino_hiptmair): face stars and NedTwo edge-star potentials
    (NedTwo_p for RT_p, NedTwo_{p+1} for BDM_p) whose local matrices carry the
    regularising mass.  The library inverts them explicitly, the oracle
    solves with their Cholesky factors.  Their condition numbers are 1e9-1e11
    (printed), but the ill-conditioned directions are the NedTwo gradients,
    the kernel of the curl map G: the right-hand sides G^T r are orthogonal
    to it and z = G y removes it, so the rounding that the small eigenvalues
    amplify stays out of z.  Hence the usual comparator bar: apply_P within
    1e-10 of the oracle's (measured 5e-15 to 3e-14); the solve meets the true
    residual 1e-10 and takes the oracle's iteration count within one."""
    d, fam, p, n, jit = case
    top, A, P, prob = setup_case(d, fam, p, n, jit, form, pc)
    rho = prob.pc_weights()
    if pc == "hybrid":
        assert abs(rho[1] / P.rho_Gamma - 1) <= 1e-8
    r = load_vectors(top.n_dofs, 41)[:, 0]
    zt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt)
    torch.cuda.synchronize()
    ref = P.apply(r)
    err = np.abs(zt.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"{fam}{p} {form} {pc}: apply_P rel err {err:.2e}, kappa_pc {_kappa_pc(P):.2e}", flush=True)
    assert err <= 1e-10
    b = load_vectors(top.n_dofs, 42)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-12)
    xo, io = pcg(lambda v: A @ v, P.apply, b, rtol=1e-12)
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info["iterations"], io["iterations"])
    assert np.linalg.norm(b - A @ xt.cpu().numpy()) <= 1e-10 * np.linalg.norm(b)


def test_hdiv_hiptmair_refuses_dirichlet():
    from paper_2506_17406_amd import rz
    X, C = kuhn_mesh(1, 3, jitter=0.1, seed=13)
    flags = np.zeros((len(C), 4), dtype=np.uint8)
    for c in range(len(C)):
        for j in range(4):
            if np.all(np.isclose(X[np.delete(C[c], j)][:, 0], 0.0)):
                flags[c, j] = 1
    with pytest.raises(rz.RzError) as e:
        rz.Problem(X, C, 2, "RT", decomposition="hiptmair", dirichlet_facet=flags)
    assert e.value.code == -2
