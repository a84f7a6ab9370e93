"""GPU checks at the benchmark's full size and launch configuration (the
jittered 8^3x6 Kuhn mesh of bench.py, p = 6 and 8): the oracle computes
sampled outputs one by one, and properties that hold at any size.

* apply_A: sampled rows (A x)_i from the oracle's stacked reference form
  (itself pinned to the direct definition) within 1e-12 max |y|;
* apply_P: symmetry r1.P^{-1}r2 = r2.P^{-1}r1, positivity, linearity --
  1e-12 relative for the additive form; 1e-10 for the hybrid sweep, whose
  result passes through four operator applies (FP64 atomic scatter in a
  varying order), so rounding breaks exact symmetry and linearity at a few
  1e-12;
* solve: the library's recursive residual <= 1e-10 and the oracle's residual
  rows b_i - (A x)_i of the returned x within 2e-10 ||b||_2 (each entry of a
  vector is bounded by its 2-norm).
* additive apply_P at p = 8 (the patch sets of 0.8-2.1 GB that stream with
  non-temporal loads): sampled outputs z_i of the oracle's additive
  preconditioner -- point-Jacobi, every patch (and H(curl) vertex
  potential) that contains dof i solved densely, and the exact coarse
  solve -- within 1e-10 max |z|.
* the mixed-precision, multi-RHS and uneven-batch workloads at their full
  size (Ned_6 on 16^3 x 6 cells in FP32 refinement and with the bfloat16
  preconditioner; RT_5 on 12^3 x 6 cells with 64 right-hand sides; the
  batch's CG_10 16^3 x 6 and Ned_10 10^3 x 6 members; the spaces leg's 2D
  Ned_6 and RT_6 on 96^2 x 2 triangles with the W^1 V-cycle, NedTwo_4 and
  BDM_4 on 8^3 x 6): the oracle's sampled residual rows of the returned
  solutions within 2e-10 ||b||_2, and the sampled estimate
  sqrt(n / |S| sum_S res_i^2) / ||b|| of the relative true residual printed.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import scipy.linalg as sla

from oracle.element import element
from oracle.mesh import Topology
from oracle.operator import cell_weights, reference_stack
from oracle.precond import interior_dofs, patch_lists, potential_patches, whitney_dofs
from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

pytestmark = pytest.mark.gpu

FULL = [("CG", 8), ("Ned", 6), ("Ned", 8), ("RT", 8)]
_cache = {}


def setup_full(fam, p, pc="hybrid"):
    if (fam, p, pc) not in _cache:
        from paper_2506_17406_amd import rz
        X, C = kuhn_mesh(8, 3, jitter=0.1, seed=2)
        el = element(3, fam, p)
        top = Topology(X, C, el)
        prob = rz.Problem(X, C, p, fam, pc=pc)
        assert prob.n_dofs == top.n_dofs
        _cache[(fam, p, pc)] = (el, top, reference_stack(el), prob)
    return _cache[(fam, p, pc)]


def sample_dofs(top, per_block=12, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for l in range(len(top.offset) - 1):
        lo, hi = top.offset[l], top.offset[l + 1]
        if hi > lo:
            out += list(rng.choice(np.arange(lo, hi), size=min(per_block, hi - lo), replace=False))
    return np.array(out)


def oracle_rows(el, top, R, x, rows):
    y = np.zeros(len(rows))
    for k, i in enumerate(rows):
        cells, locs = np.nonzero(top.cell_dofs == i)
        for c, loc in zip(cells, locs):
            w = cell_weights(el, top.coords[top.cells[c]])
            y[k] += np.einsum("q,qj,j->", w, R[:, loc, :], x[top.cell_dofs[c]])
    return y


@pytest.mark.parametrize("fam,p", FULL)
def test_apply_A_sampled(fam, p):
    el, top, R, prob = setup_full(fam, p)
    x = load_vectors(top.n_dofs, 5)[:, 0]
    yt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_A(torch.from_numpy(x).cuda(), yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    rows = sample_dofs(top)
    ref = oracle_rows(el, top, R, x, rows)
    assert np.abs(y[rows] - ref).max() <= 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("pc", ["additive", "hybrid"])
@pytest.mark.parametrize("fam,p", FULL)
def test_apply_P_properties(fam, p, pc):
    el, top, R, prob = setup_full(fam, p, pc)
    tol = 1e-12 if pc == "additive" else 1e-10
    r = load_vectors(top.n_dofs, 8, n_rhs=2)
    rt = torch.from_numpy(np.ascontiguousarray(r.T)).cuda()
    z1, z2, z3 = (torch.empty(top.n_dofs, dtype=torch.float64, device="cuda") for _ in range(3))
    prob.apply_P(rt[0].contiguous(), z1)
    prob.apply_P(rt[1].contiguous(), z2)
    prob.apply_P((rt[0] + 2.0 * rt[1]).contiguous(), z3)
    torch.cuda.synchronize()
    a = float(torch.dot(rt[0], z2))
    b = float(torch.dot(rt[1], z1))
    assert abs(a - b) <= tol * max(abs(a), abs(b))
    assert float(torch.dot(rt[0], z1)) > 0 and float(torch.dot(rt[1], z2)) > 0
    lin = z1 + 2.0 * z2
    assert float((z3 - lin).abs().max()) <= tol * float(lin.abs().max())


@pytest.mark.parametrize("fam,p", FULL)
def test_solve_sampled_residual(fam, p):
    el, top, R, prob = setup_full(fam, p)
    b = load_vectors(top.n_dofs, 3)[:, 0]
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    info = prob.solve(bt, xt, rtol=1e-10)
    assert info["rel_residual"] <= 1e-10
    x = xt.cpu().numpy()
    rows = sample_dofs(top, seed=1)
    res = b[rows] - oracle_rows(el, top, R, x, rows)
    assert np.abs(res).max() <= 2e-10 * np.linalg.norm(b)


# ---- sampled outputs of the additive preconditioner at p = 8 ---------------
def dof_cells(top):
    """For every dof: the cells containing it and its local index there."""
    flat = top.cell_dofs.ravel()
    order = np.argsort(flat, kind="stable")
    ptr = np.searchsorted(flat[order], np.arange(top.n_dofs + 1))
    return order, ptr


def cell_matrix_stacked(el, top, R, c):
    return np.tensordot(cell_weights(el, top.coords[top.cells[c]]), R, axes=1)


def local_matrix(el, top, R, dc, idx):
    """A[idx][:, idx] summed from the cells that hold any of the dofs idx."""
    order, ptr = dc
    cells = sorted({int(order[k]) // el.n for i in idx for k in range(ptr[i], ptr[i + 1])})
    pos = {int(i): a for a, i in enumerate(idx)}
    Ap = np.zeros((len(idx), len(idx)))
    for c in cells:
        loc = [(a, pos[int(g)]) for a, g in enumerate(top.cell_dofs[c]) if int(g) in pos]
        la = np.array([a for a, _ in loc])
        pa = np.array([b for _, b in loc])
        Ap[np.ix_(pa, pa)] += cell_matrix_stacked(el, top, R, c)[np.ix_(la, la)]
    return Ap


def sampled_additive_apply(el, top, R, fam, r, rows):
    """z_i (i in rows) of P^{-1} r = D_I^{-1} r_I + sum_m R_m^T A_m^{-1} R_m r
    + R_W^T A_W^{-1} R_W r (Sec. 6; the oracle's additive form), computing
    only the patches that contain a sampled dof."""
    dc = dof_cells(top)
    k = {"CG": 0, "Ned": 1, "RT": 2}[fam]
    z = np.zeros(len(rows))
    where = {int(i): a for a, i in enumerate(rows)}
    # interior point-Jacobi
    I0 = interior_dofs(top)[0] if top.n_interior else top.n_dofs
    for i, a in where.items():
        if i >= I0:
            c_cell = dc[0][dc[1][i]] // el.n
            loc = list(top.cell_dofs[c_cell]).index(i)
            z[a] += r[i] / cell_matrix_stacked(el, top, R, c_cell)[loc, loc]
    # patches containing a sampled dof
    for idx in patch_lists(top, fam):
        hit = [i for i in idx if int(i) in where]
        if not hit:
            continue
        y = sla.cho_solve(sla.cho_factor(local_matrix(el, top, R, dc, idx), lower=True), r[idx])
        for i in hit:
            z[where[int(i)]] += y[int(np.searchsorted(idx, i))]
    if fam == "Ned":
        p = el.p
        cg_N = (1, p - 1, (p - 1) * (p - 2) // 2, (p - 1) * (p - 2) * (p - 3) // 6)
        for G in potential_patches(top, cg_N):
            G = G.tocsr()
            S = np.flatnonzero(np.diff(G.indptr))          # rows the potential touches
            hit = [i for i in S if int(i) in where]
            if not hit:
                continue
            GS = G[S].toarray()
            AV = GS.T @ local_matrix(el, top, R, dc, S) @ GS
            y = GS @ sla.cho_solve(sla.cho_factor(AV, lower=True), GS.T @ r[S])
            for i in hit:
                z[where[int(i)]] += y[int(np.searchsorted(S, i))]
    # exact coarse solve on the Whitney dofs
    W = whitney_dofs(top, k)
    wpos = {int(w): a for a, w in enumerate(W)}
    wloc = [a for a, g in enumerate(top.cell_dofs[0]) if int(g) in wpos]
    AW = np.zeros((len(W), len(W)))
    Rw = R[:, wloc][:, :, wloc]
    for c in range(top.n_cells):
        g = np.array([wpos[int(top.cell_dofs[c][a])] for a in wloc])
        AW[np.ix_(g, g)] += np.tensordot(cell_weights(el, top.coords[top.cells[c]]), Rw, axes=1)
    zW = sla.cho_solve(sla.cho_factor(AW, lower=True), r[W])
    for i, a in where.items():
        if i in wpos:
            z[a] += zW[wpos[i]]
    return z


@pytest.mark.parametrize("fam", ["CG", "Ned", "RT"])
def test_additive_apply_P_sampled(fam):
    el, top, R, prob = setup_full(fam, 8, "additive")
    r = load_vectors(top.n_dofs, 12)[:, 0]
    zt = torch.empty(top.n_dofs, dtype=torch.float64, device="cuda")
    prob.apply_P(torch.from_numpy(r).cuda(), zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    rows = sample_dofs(top, per_block=6, seed=4)
    ref = sampled_additive_apply(el, top, R, fam, r, rows)
    err = np.abs(z[rows] - ref).max() / np.abs(z).max()
    print(f"additive apply_P {fam}8 n=8: sampled max rel diff {err:.2e}", flush=True)
    assert err <= 1e-10, err


# ---- the other workloads at full size ---------------------------------------
def _residual_rows(el, top, R, b, x, rows):
    res = b[rows] - oracle_rows(el, top, R, x, rows)
    est = np.sqrt(top.n_dofs / len(rows) * np.sum(res ** 2)) / np.linalg.norm(b)
    return np.abs(res).max() / np.linalg.norm(b), est


WORKLOADS = {
    # name: (space, p, n, mesh seed, load seed, precision, columns)
    "mixed-fp32ir-Ned6-n16": ("Ned", 6, 16, 4, 5, "fp32-ir", 1),
    "mixed-bf16pc-Ned6-n16": ("Ned", 6, 16, 4, 5, "bf16-pc", 1),
    "multirhs-bf16pc-RT5-n12-64": ("RT", 5, 12, 6, 7, "bf16-pc", 64),
    "multirhs-fp32ir-RT5-n12-64": ("RT", 5, 12, 6, 7, "fp32-ir", 64),
    "batch-bf16pc-CG10-n16": ("CG", 10, 16, 128, 228, "bf16-pc", 1),
    "batch-bf16pc-Ned10-n10": ("Ned", 10, 10, 106, 206, "bf16-pc", 1),
    # the spaces leg: 2D with the W^1 V-cycle over the Kuhn meshes 96, .., 3
    # (dimension and coarse solver appended), second-kind 3D
    "spaces-Ned6-n96-2d-mg": ("Ned", 6, 96, 2, 3, "fp64", 1, 2, "mg"),
    "spaces-RT6-n96-2d-mg": ("RT", 6, 96, 2, 3, "fp64", 1, 2, "mg"),
    "spaces-NedTwo4-n8": ("NedTwo", 4, 8, 2, 3, "fp64", 1),
    "spaces-BDM4-n8": ("BDM", 4, 8, 2, 3, "fp64", 1),
}


def _hierarchy(n, d):
    out = [kuhn_mesh(n, d)]
    while n % 2 == 0 and n > 1:
        n //= 2
        out.append(kuhn_mesh(n, d))
    return out


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_workload_sampled_residual(name):
    from paper_2506_17406_amd import rz
    fam, p, n, ms, ls, prec, nc = WORKLOADS[name][:7]
    d, coarse = WORKLOADS[name][7:] if len(WORKLOADS[name]) > 7 else (3, "exact")
    print(f"workload {name}: setup", flush=True)
    X, C = kuhn_mesh(n, d, jitter=0.1, seed=ms)
    prob = rz.Problem(X, C, p, fam, precision=prec, coarse=coarse,
                      mg_meshes=_hierarchy(n, d) if coarse == "mg" else None)
    try:
        B = load_vectors(prob.n_dofs, ls, n_rhs=nc)
        Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().T if nc > 1 else torch.from_numpy(B[:, 0]).cuda()
        Xt = torch.zeros_like(Bt)
        info = prob.solve(Bt, Xt, rtol=1e-10)
        torch.cuda.synchronize()
        Xs = Xt.cpu().numpy().reshape(prob.n_dofs, nc)
        infos = info if nc > 1 else [info]
    finally:
        prob.close()
        torch.cuda.empty_cache()
    el = element(d, fam, p)
    top = Topology(X, C, el)
    R = reference_stack(el)
    rows = sample_dofs(top, per_block=10, seed=2)
    worst, worst_est = 0.0, 0.0
    for j in sorted({0, nc // 3, (2 * nc) // 3, nc - 1}):
        mx, est = _residual_rows(el, top, R, B[:, j], Xs[:, j], rows)
        worst, worst_est = max(worst, mx), max(worst_est, est)
    its = [i["iterations"] for i in infos]
    print(f"workload {name}: {prob.n_dofs} dofs x {nc}, iterations {min(its)}-{max(its)}, "
          f"library residual <= {max(i['rel_residual'] for i in infos):.2e}, oracle sampled rows: "
          f"max |res_i| / ||b|| = {worst:.2e}, estimated ||res|| / ||b|| = {worst_est:.2e}", flush=True)
    assert all(i["status"] == 0 for i in infos)
    assert worst <= 2e-10
