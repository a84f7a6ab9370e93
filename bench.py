"""Benchmark: Riesz-map PCG solves to relative residual 1e-10 on one MI355X.

Workload (one step): the 3D plain-FP64 sweep -- H(grad) (CG_p), H(curl)
(Ned_p, first kind) and H(div) (RT_p) Riesz maps, alpha = beta = 1, on the
Freudenthal mesh of the unit cube with 8 cells per edge (3072 tetrahedra),
interior vertices jittered by U(-0.1h, 0.1h) (seed 2), p = 3..8, one
uniform[-1, 1] load vector per problem (seed 3), each solved from x = 0 to
||r|| <= 1e-10 ||b|| with the hybrid preconditioner.  By default the 18
problems are solved together through the batch interface (a stream per
problem); the one-after-another time is reported beside it.  Inputs are
resident in HBM before timing; setup (reference build, numbering, patch and
coarse factorisation) is timed separately.  value = total dofs solved per
step / step time.

Also reported: the operator apply (the dominant kernel by flops) against
the FP64 matrix peak and the largest patch stream of the preconditioner
against HBM bandwidth, both timed with HIP events on the launch stream; two
compact comparisons (mixed precision on H(curl) Ned_6 16^3x6 to a true
FP64 residual of 1e-10, and 64 right-hand sides on H(div) RT_5 12^3x6
batched against one by one); and the oracle (plain NumPy/SciPy FP64) timed
on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--degrees", type=str, default="3,4,5,6,7,8")
    ap.add_argument("--spaces", type=str, default="CG,Ned,RT")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--sweep-mode", choices=["batched", "sequential"], default="batched",
                    help="sweep step: the 18 problems solved one after another, or together as one batch "
                         "(a stream per problem, captured iteration graphs)")
    ap.add_argument("--workload", choices=["sweep", "multirhs", "mixed", "batch", "decompositions", "hodge", "spaces"],
                    default="sweep",
                    help="sweep: the 3D FP64 sweep (default, the headline line); multirhs: H(div) RT_5 on the "
                         "12^3x6 mesh with 64 right-hand sides, one batched solve vs 64 single solves; mixed: "
                         "H(curl) Ned_6 on the 16^3x6 mesh, FP32 refinement and FP32/BF16-stored preconditioners vs "
                         "plain FP64 PCG; batch: 32 uneven "
                         "H(grad)/H(curl) problems solved together vs one by one; decompositions: the default "
                         "split solvers against the vertex-star comparators PAFW(0)(X^k_Gamma)+J and "
                         "PAFW(0)(X^k) and the Hiptmair-Toselli forms on the sweep mesh (--degrees, default 4,5 "
                         "for this workload); hodge: the Hodge Laplacians on the Fichera corner with MINRES; "
                         "spaces: 2D H(curl)/H(div) and the second-kind 3D spaces")
    ap.add_argument("--batch-count", type=int, default=32)
    ap.add_argument("--batch-max-gb", type=float, default=240.0)
    ap.add_argument("--batch-precision", choices=["fp64", "fp32-pc", "bf16-pc"], default="bf16-pc")
    ap.add_argument("--batch-no-fp64", action="store_true",
                    help="skip the plain FP64 batch run that the reduced-precision batch is compared with")
    ap.add_argument("--inner-rtol", type=float, default=0.0)
    ap.add_argument("--pc", choices=["hybrid", "additive"], default="hybrid",
                    help="preconditioner form: the symmetric multiplicative hybrid of the paper's experiments "
                         "(default) or the additive Schwarz form")
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--multirhs-modes", type=str, default="fp64,fp32-ir,bf16-pc",
                    help="precision modes timed by the multirhs workload (fp64 always runs)")
    ap.add_argument("--no-legs", action="store_true",
                    help="sweep workload: skip the compact mixed-precision (Ned_6 16^3x6), 64-column (RT_5 "
                         "12^3x6), Hodge-Laplacian (p = 4, Fichera corner) and 2D / second-kind spaces legs "
                         "that the default line carries")
    ap.add_argument("--leg-steps", type=int, default=3)
    ap.add_argument("--profile-copy-bytes", type=int, default=0,
                    help="after the measurement, one plain device copy of this many bytes (a known-size kernel "
                         "that calibrates HBM counters in profiler runs)")
    return ap.parse_args()


def multirhs(args):
    """H(div) RT_5 on the jittered 12^3x6 = 10368-tet mesh (mesh seed 6), 64
    uniform[-1,1] right-hand sides drawn in sequence (seed 7), all solved to
    1e-10: one batched solve of the 64 columns vs the 64 columns one by one
    (FP64), and the batched solve in each precision mode of --multirhs-modes;
    value = the fastest mode whose largest true FP64 residual meets 1.2e-10."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    torch.cuda.set_device(0)
    X, C = kuhn_mesh(12, 3, jitter=0.1, seed=6)
    t0 = time.perf_counter()
    prob = rz.Problem(X, C, 5, "RT", pc=args.pc)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nr = args.nrhs
    B = torch.from_numpy(np.ascontiguousarray(load_vectors(prob.n_dofs, 7, n_rhs=nr).T)).cuda().T
    X_ = torch.zeros_like(B)
    Y_ = torch.empty_like(B)
    print(f"setup RT5 n=12: {prob.n_dofs} dofs x {nr} rhs in {t_setup:.1f}s", file=sys.stderr, flush=True)

    def batched(pr):
        for _ in range(args.warmup):
            X_.zero_()
            pr.solve(B, X_, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            X_.zero_()
            infos = pr.solve(B, X_, rtol=1e-10)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        prob.apply_A(X_, Y_)  # true residuals under the FP64 operator
        res = float(((B - Y_).norm(dim=0) / B.norm(dim=0)).max())
        its = [i["iterations"] for i in infos]
        out = {"value": prob.n_dofs * nr / dt, "ms": dt * 1e3, "iterations": {"min": min(its), "max": max(its)},
               "max_true_rel_residual": res}
        if any(i.get("outer_iterations", 0) for i in infos):
            out["outer_iterations"] = max(i["outer_iterations"] for i in infos)
        print(f"{nr} columns: {dt * 1e3:.1f} ms, {min(its)}-{max(its)} its, true residual <= {res:.2e}",
              file=sys.stderr, flush=True)
        return out

    modes = {"fp64": batched(prob)}
    # the same columns one at a time (FP64)
    xs = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_its = []
    for j in range(nr):
        xs.zero_()
        seq_its.append(prob.solve(B[:, j].contiguous(), xs, rtol=1e-10)["iterations"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for m in [m for m in args.multirhs_modes.split(",") if m and m != "fp64"]:
        pr = rz.Problem(X, C, 5, "RT", pc=args.pc, precision=m)
        torch.cuda.synchronize()
        print(f"mode {m}:", file=sys.stderr, flush=True)
        modes[m] = batched(pr)
        pr.close()
        torch.cuda.empty_cache()
    ok = [m for m in modes if modes[m]["max_true_rel_residual"] <= 1.2e-10]
    best = min(ok, key=lambda m: modes[m]["ms"]) if ok else "fp64"
    dt = modes[best]["ms"] / 1e3
    line = {
        "metric": "Riesz-map solve DOFs/s to rel. residual 1e-10 (multi-RHS)",
        "value": prob.n_dofs * nr / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32-ir": "f32 applies, f64 refinement",
                                       "fp32-pc": "f64 operator, f32-stored preconditioner",
                                       "bf16-pc": "f64 operator, bf16-stored preconditioner"}[best],
        "data": "synthetic",
        "config": {"workload": f"H(div) RT_5 Riesz map, jittered Kuhn 12^3x6 = 10368 tets, {nr} right-hand sides "
                               f"solved together, rtol 1e-10", "dofs": prob.n_dofs, "n_rhs": nr, "preconditioner": args.pc,
                   "mode": best, "setup_s": round(t_setup, 2)},
        "modes": modes,
        "sequential": {"value": prob.n_dofs * nr / t_seq, "seconds": t_seq,
                       "iterations": {"min": min(seq_its), "max": max(seq_its)}},
        "speedup_vs_sequential_fp64": t_seq / dt,
        "speedup_vs_fp64_batched": modes["fp64"]["ms"] / (dt * 1e3),
    }
    print(json.dumps(line), flush=True)


def _apply_time(fn, x, y, reps, stream):
    import torch
    for _ in range(3):
        fn(x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        fn(x, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3 / reps


def mixed(args):
    """H(curl) Ned_6 on the jittered 16^3x6 = 24576-tet mesh (mesh seed 4),
    one uniform[-1,1] load vector (seed 5), solved to a true FP64 relative
    residual of 1e-10 by FP32 iterative refinement, against plain FP64 PCG
    on the same GPU."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    X, C = kuhn_mesh(16, 3, jitter=0.1, seed=4)
    t0 = time.perf_counter()
    pm = rz.Problem(X, C, 6, "Ned", precision="fp32-ir", inner_rtol=args.inner_rtol, pc=args.pc)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"setup Ned6 n=16 (FP64 + FP32 copies): {pm.n_dofs} dofs in {t_setup:.1f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    p64 = rz.Problem(X, C, 6, "Ned", pc=args.pc)
    torch.cuda.synchronize()
    t_set64 = time.perf_counter() - t0
    # the W^1 multigrid V-cycle over the Kuhn meshes 16, 8, 4, 2, 1 in place
    # of the dense coarse inverse
    t0 = time.perf_counter()
    pmg = rz.Problem(X, C, 6, "Ned", pc=args.pc, coarse="mg", mg_meshes=[kuhn_mesh(m, 3) for m in (16, 8, 4, 2, 1)])
    torch.cuda.synchronize()
    t_setmg = time.perf_counter() - t0
    ppc = rz.Problem(X, C, 6, "Ned", precision="fp32-pc", pc=args.pc)
    pbf = rz.Problem(X, C, 6, "Ned", precision="bf16-pc", pc=args.pc)
    torch.cuda.synchronize()
    print("setup FP64, FP32- and BF16-preconditioner handles done", file=sys.stderr, flush=True)
    b = torch.from_numpy(load_vectors(pm.n_dofs, 5)[:, 0]).cuda()
    xm, x64, xpc, xbf = torch.zeros_like(b), torch.zeros_like(b), torch.zeros_like(b), torch.zeros_like(b)
    xmg = torch.zeros_like(b)

    def timed(prob, x):
        for _ in range(args.warmup):
            x.zero_()
            prob.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            info = prob.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, info

    dt_m, info_m = timed(pm, xm)
    print(f"FP32-IR: {dt_m * 1e3:.1f} ms, {info_m['iterations']} its, {info_m['outer_iterations']} outer",
          file=sys.stderr, flush=True)
    dt_64, info_64 = timed(p64, x64)
    print(f"FP64: {dt_64 * 1e3:.1f} ms, {info_64['iterations']} its", file=sys.stderr, flush=True)
    dt_pc, info_pc = timed(ppc, xpc)
    print(f"FP32 preconditioner: {dt_pc * 1e3:.1f} ms, {info_pc['iterations']} its", file=sys.stderr, flush=True)
    dt_bf, info_bf = timed(pbf, xbf)
    print(f"BF16 preconditioner: {dt_bf * 1e3:.1f} ms, {info_bf['iterations']} its", file=sys.stderr, flush=True)
    dt_mg, info_mg = timed(pmg, xmg)
    print(f"FP64 with the W^1 V-cycle: {dt_mg * 1e3:.1f} ms, {info_mg['iterations']} its, setup {t_setmg:.2f} s "
          f"(dense coarse inverse: {t_set64:.2f} s)", file=sys.stderr, flush=True)
    # true FP64 residuals and the distance between the solutions
    r = torch.empty_like(b)
    nb = b.norm().item()

    def true_res(x):
        p64.apply_A(x, r)
        return (b - r).norm().item() / nb

    res64, res_m, res_pc, res_bf = true_res(x64), true_res(xm), true_res(xpc), true_res(xbf)
    res_mg = true_res(xmg)
    diff = (xm - x64).norm().item() / x64.norm().item()
    diff_pc = (xpc - x64).norm().item() / x64.norm().item()
    diff_bf = (xbf - x64).norm().item() / x64.norm().item()
    # dominant kernels: the FP32 and FP64 operator applies, the two preconditioner applies
    xa = torch.rand(pm.n_dofs, dtype=torch.float64, device="cuda")
    ya = torch.empty_like(xa)
    reps = args.apply_reps
    t_a32 = _apply_time(lambda u, v: pm.apply_A(u, v, fp32=True), xa, ya, reps, stream)
    t_a64 = _apply_time(pm.apply_A, xa, ya, reps, stream)
    t_p32 = _apply_time(lambda u, v: pm.apply_P(u, v, fp32=True), xa, ya, reps, stream)
    t_p64 = _apply_time(pm.apply_P, xa, ya, reps, stream)
    t_pbf = _apply_time(lambda u, v: pbf.apply_P(u, v, fp32=True), xa, ya, reps, stream)
    flops = 2.0 * pm.Q * pm.n_loc ** 2 * pm.n_cells
    tf32 = flops / t_a32 / 1e12
    # the fastest mode whose true residual meets the target
    modes = [("bf16-pc", dt_bf, res_bf), ("fp32-pc", dt_pc, res_pc), ("fp32-ir", dt_m, res_m)]
    mode, dt_best, _ = min((m for m in modes if m[2] <= 1.2e-10), key=lambda m: m[1], default=modes[1])
    best_pc = mode != "fp32-ir"
    line = {
        "metric": "Riesz-map solve DOFs/s to rel. residual 1e-10 (mixed precision)",
        "value": pm.n_dofs / dt_best, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt_best * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16-pc": "f64 operator, bf16-stored preconditioner",
                  "fp32-pc": "f64 operator, f32-stored preconditioner",
                  "fp32-ir": "f32 applies, f64 refinement"}[mode],
        "data": "synthetic",
        "config": {"workload": "H(curl) Ned_6 Riesz map, jittered Kuhn 16^3x6 = 24576 tets, mixed precision to "
                               "true FP64 rel. residual 1e-10", "dofs": pm.n_dofs,
                   "mode": mode, "preconditioner": args.pc,
                   "setup_s": round(t_setup, 2)},
        "roofline": ({"kernel": "apply_A FP64 (Ned6)", "bound": "mfma", "achieved": flops / t_a64 / 1e12,
                      "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": flops / t_a64 / 1e12 / PEAK_FP64_TFLOPS,
                      "traffic": None, "flops_per_launch": flops, "launch_us": t_a64 * 1e6} if best_pc else
                     {"kernel": "apply_A FP32 (Ned6)", "bound": "mfma", "achieved": tf32, "peak": PEAK_FP32_TFLOPS,
                      "unit": "TFLOP/s", "frac": tf32 / PEAK_FP32_TFLOPS, "traffic": None,
                      "flops_per_launch": flops, "launch_us": t_a32 * 1e6}),
        "bf16_pc": {"value": pm.n_dofs / dt_bf, "ms": dt_bf * 1e3, "iterations": info_bf["iterations"],
                    "true_rel_residual": res_bf, "rel_diff_vs_fp64_solution": diff_bf},
        "fp64_mg": {"value": pm.n_dofs / dt_mg, "ms": dt_mg * 1e3, "iterations": info_mg["iterations"],
                    "true_rel_residual": res_mg, "setup_s": round(t_setmg, 2),
                    "setup_s_dense_coarse": round(t_set64, 2)},
        "fp32_pc": {"value": pm.n_dofs / dt_pc, "ms": dt_pc * 1e3, "iterations": info_pc["iterations"],
                    "true_rel_residual": res_pc, "rel_diff_vs_fp64_solution": diff_pc},
        "fp32_ir": {"value": pm.n_dofs / dt_m, "ms": dt_m * 1e3, "iterations": info_m["iterations"],
                    "outer_iterations": info_m["outer_iterations"], "true_rel_residual": res_m,
                    "rel_diff_vs_fp64_solution": diff},
        "fp64": {"value": pm.n_dofs / dt_64, "ms": dt_64 * 1e3, "iterations": info_64["iterations"],
                 "true_rel_residual": res64},
        "speedup_vs_fp64": dt_64 / dt_best,
        "apply_us": {"A_fp32": t_a32 * 1e6, "A_fp64": t_a64 * 1e6, "P_fp32": t_p32 * 1e6, "P_fp64": t_p64 * 1e6,
                     "P_bf16": t_pbf * 1e6},
    }
    print(json.dumps(line), flush=True)


def _batch_bytes(sp, n, p):
    """Device bytes of one problem, from the largest-patch sizes (interior
    stars; boundary stars are smaller): FP64 + FP32 patch and coarse
    inverses, tables and about 16 work vectors."""
    V, E, F, C = (n + 1) ** 3, 7 * n ** 3 + 9 * n ** 2 + 3 * n, 12 * n ** 3 + 6 * n ** 2, 6 * n ** 3
    mv = 1 + 14 * (p - 1) + 18 * (p - 1) * (p - 2)
    if sp == "CG":
        dofs = V + E * (p - 1) + F * (p - 1) * (p - 2) // 2 + C * (p - 1) * (p - 2) * (p - 3) // 6
        patches, nW = V * mv * mv / 2, V
    else:
        me = 1 + 3 * (p - 1) * (p + 2)
        dofs = p * E + F * (p - 1) * p + C * (p - 1) * (p - 2) * (p + 1) // 2
        patches, nW = V * mv * mv / 2 + E * me * me / 2, E
    return 12.0 * (patches + nW * nW / 2) + 16 * 8 * dofs, dofs


def batch_workload(args):
    """The uneven batch: 32 H(grad)/H(curl) problems with n in 4..16 and p
    in 2..10 drawn from default_rng(8) (a draw is redrawn while the batch
    would exceed the memory budget), jittered Kuhn meshes (seed 100 + i),
    load vectors seed 200 + i, solved together to 1e-10 with captured
    iteration graphs, against the same problems solved one by one and the
    same batch with plain FP64 handles."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors, uneven_batch
    torch.cuda.set_device(0)
    draws, rng = uneven_batch(8, args.batch_count)
    budget = args.batch_max_gb * 1e9
    while sum(_batch_bytes(d[0], d[1], d[2])[0] for d in draws) > budget:
        # redraw the largest problem from the continuing generator
        j = max(range(len(draws)), key=lambda k: _batch_bytes(*draws[k][:3])[0])
        sp = ("CG", "Ned")[int(rng.integers(2))]
        draws[j] = (sp, int(rng.integers(4, 17)), int(rng.integers(2, 11)), draws[j][3], draws[j][4])
    probs, bs, xs = [], [], []
    t0 = time.perf_counter()
    for sp, n, p, ms, rs in draws:
        X, C = kuhn_mesh(n, 3, jitter=0.1, seed=ms)
        t1 = time.perf_counter()
        prob = rz.Problem(X, C, p, sp, pc=args.pc, precision=args.batch_precision)
        torch.cuda.synchronize()
        probs.append(prob)
        bs.append(torch.from_numpy(load_vectors(prob.n_dofs, rs)[:, 0]).cuda())
        xs.append(torch.zeros_like(bs[-1]))
        print(f"setup {sp}{p} n={n}: {prob.n_dofs} dofs in {time.perf_counter() - t1:.1f}s", file=sys.stderr,
              flush=True)
    t_setup = time.perf_counter() - t0
    total = sum(p.n_dofs for p in probs)
    t1 = time.perf_counter()
    B = rz.Batch(probs)
    t_tune = time.perf_counter() - t1
    for _ in range(args.warmup):
        for x in xs:
            x.zero_()
        B.solve(bs, xs, rtol=1e-10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for x in xs:
            x.zero_()
        infos = B.solve(bs, xs, rtol=1e-10)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    print(f"batch: {dt * 1e3:.1f} ms for {total} dofs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq = []
    for prob, b, x in zip(probs, bs, xs):
        x.zero_()
        seq.append(prob.solve(b, x, rtol=1e-10)["iterations"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    print(f"one by one: {t_seq * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # the plain FP64 reference: the same problems as an FP64 batch (the
    # reduced-precision handles are released first)
    fp64 = None
    if args.batch_precision != "fp64" and not args.batch_no_fp64:
        B.close()
        for prob in probs:
            prob.close()
        probs = []
        torch.cuda.empty_cache()
        for sp, n, p, ms, rs in draws:
            X, C = kuhn_mesh(n, 3, jitter=0.1, seed=ms)
            probs.append(rz.Problem(X, C, p, sp, pc=args.pc))
        torch.cuda.synchronize()
        B64 = rz.Batch(probs)
        for x in xs:
            x.zero_()
        B64.solve(bs, xs, rtol=1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            for x in xs:
                x.zero_()
            infos64 = B64.solve(bs, xs, rtol=1e-10)
        torch.cuda.synchronize()
        dt64 = (time.perf_counter() - t1) / args.steps
        print(f"FP64 batch: {dt64 * 1e3:.1f} ms", file=sys.stderr, flush=True)
        fp64 = {"value": total / dt64, "ms": dt64 * 1e3,
                "iterations": {"min": min(i["iterations"] for i in infos64),
                               "max": max(i["iterations"] for i in infos64)},
                "max_rel_residual": max(i["rel_residual"] for i in infos64)}
    line = {
        "metric": "Riesz-map solve DOFs/s to rel. residual 1e-10 (uneven batch)",
        "value": total / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32-pc": "f64 operator, f32-stored preconditioner",
                  "bf16-pc": "f64 operator, bf16-stored preconditioner", "fp64": "f64"}[args.batch_precision],
        "data": "synthetic",
        "config": {"workload": f"uneven batch of {len(probs)} H(grad)/H(curl) Riesz maps, n in 4..16, p in 2..10, "
                               "jittered Kuhn meshes, rtol 1e-10", "total_dofs": total,
                   "problems": [f"{d[0]}{d[2]} n={d[1]}" for d in draws], "preconditioner": args.pc,
                   "setup_s": round(t_setup, 1), "tune_s": round(t_tune, 2)},
        "iterations": {"min": min(i["iterations"] for i in infos), "max": max(i["iterations"] for i in infos)},
        "max_rel_residual": max(i["rel_residual"] for i in infos),
        "sequential": {"value": total / t_seq, "seconds": t_seq},
        "speedup_vs_sequential": t_seq / dt,
        "fp64_batch": fp64,
        "speedup_vs_fp64_batch": fp64["ms"] / (dt * 1e3) if fp64 else None,
    }
    print(json.dumps(line), flush=True)


def decompositions(args):
    """The space decompositions of Sec. 6 side by side on the sweep's mesh
    (jittered 8^3x6, mesh seed 2, load seed 3), FP64 PCG to 1e-10: the
    default split solvers, the vertex-star split PAFW(0)(X^k_Gamma)+J, the
    full vertex stars PAFW(0)(X^k), the defaults without the split
    (H(curl) PH(X^0, X^{1,I}), H(div) PAFW(1)(X^2)), for H(curl) the
    standard Hiptmair-Toselli PH(X^0_Gamma, X^1_Gamma)+J and PH(X^0, X^1),
    and for H(div) the type-I Hiptmair-Toselli PH(X^{1,I}_Gamma,
    X^{2,I}_Gamma)+J and PH(X^{1,I}, X^{2,I}) and the standard one
    PH(X^1_Gamma, X^2_Gamma)+J and PH(X^1, X^2) (NedTwo potentials with the
    regularising mass).
    Per problem: setup, iterations, solve time, patch sizes.  Roofline: the additive full-star
    preconditioner apply of the largest problem, an HBM stream of the packed
    patch and coarse inverses."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    X, C = kuhn_mesh(args.n, 3, jitter=0.1, seed=2)
    spaces = args.spaces.split(",")
    degrees = [4, 5] if args.degrees == "3,4,5,6,7,8" else [int(p) for p in args.degrees.split(",")]
    forms_of = {"CG": ["paper", "vertex", "vertex-full"],
                "Ned": ["paper", "paper-full", "hiptmair", "hiptmair-full", "vertex", "vertex-full"],
                "RT": ["paper", "paper-full", "typeI", "typeI-full", "hiptmair", "hiptmair-full", "vertex",
                       "vertex-full"]}
    forms = ["paper", "vertex", "vertex-full", "paper-full", "hiptmair", "hiptmair-full", "typeI", "typeI-full"]
    # Whitney (coarse) dof counts: vertices, edges or faces of the mesh
    Cs = np.sort(C, axis=1)
    n_sub = {0: X.shape[0],
             1: len(np.unique(Cs[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]].reshape(-1, 2), axis=0)),
             2: len(np.unique(Cs[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=0))}
    rows, tot = [], {f: [0, 0.0, []] for f in forms}
    for fam in spaces:
        for p in degrees:
            for form in forms_of[fam]:
                t0 = time.perf_counter()
                prob = rz.Problem(X, C, p, fam, pc=args.pc, decomposition=form)
                torch.cuda.synchronize()
                t_set = time.perf_counter() - t0
                b = torch.from_numpy(load_vectors(prob.n_dofs, 3)[:, 0]).cuda()
                x = torch.zeros_like(b)
                for _ in range(args.warmup):
                    x.zero_()
                    prob.solve(b, x, rtol=1e-10)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    x.zero_()
                    info = prob.solve(b, x, rtol=1e-10)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / args.steps
                sets = prob.patch_sets()
                m = np.array([st["max_size"] for st in sets])
                packed = sum(st["packed_entries"] for st in sets)
                t_p = _apply_time(prob.apply_P, b, x, args.apply_reps, stream)
                rows.append(dict(space=fam, p=p, decomposition=form, dofs=prob.n_dofs, its=info["iterations"],
                                 rel_res=info["rel_residual"], cond=round(info["cond_estimate"], 3),
                                 solve_ms=round(dt * 1e3, 3), apply_P_us=round(t_p * 1e6, 1),
                                 setup_s=round(t_set, 2), max_patch=int(m.max()),
                                 patch_mb=round(float(packed) * 8 / 1e6, 1)))
                tot[form][0] += prob.n_dofs
                tot[form][1] += dt
                if fam not in tot[form][2]:
                    tot[form][2].append(fam)
                print(f"{fam}{p} {form}: {prob.n_dofs} dofs, setup {t_set:.2f}s, {info['iterations']} its, "
                      f"{dt * 1e3:.1f} ms, apply_P {t_p * 1e6:.0f} us, max patch {m.max()}", file=sys.stderr,
                      flush=True)
                prob.close()
                del prob
                torch.cuda.empty_cache()
    # roofline: additive full-star apply_P of the largest problem
    big = max((r for r in rows if r["decomposition"] == "vertex-full"), key=lambda r: r["patch_mb"])
    prob = rz.Problem(X, C, big["p"], big["space"], pc="additive", decomposition="vertex-full")
    ptr, _ = rz.patch_lists(X, C, big["p"], big["space"], "vertex-full")
    m = np.diff(ptr).astype(np.float64)
    nW = n_sub[{"CG": 0, "Ned": 1, "RT": 2}[big["space"]]]
    # packed patch inverses, packed coarse inverse, r read and z written
    nbytes = 8.0 * ((m * (m + 1) / 2).sum() + nW * (nW + 1) / 2 + 2 * prob.n_dofs)
    r = torch.from_numpy(load_vectors(prob.n_dofs, 3)[:, 0]).cuda()
    z = torch.empty_like(r)
    t_add = _apply_time(prob.apply_P, r, z, args.apply_reps, stream)
    gbs = nbytes / t_add / 1e9
    d_paper, d_full = tot["paper"], tot["vertex-full"]
    line = {
        "metric": "Riesz-map solve DOFs/s to rel. residual 1e-10 (decomposition comparison)",
        "value": d_paper[0] / d_paper[1], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": d_paper[1] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Sec. 6 decompositions: {'/'.join(spaces)} x p={','.join(map(str, degrees))} on the "
                               f"jittered Kuhn {args.n}^3x6 mesh, rtol 1e-10, {args.pc} preconditioner; value is the "
                               "default split solvers, the comparators beside it",
                   "preconditioner": args.pc},
        "per_decomposition": {f: {"spaces": tot[f][2], "dofs": tot[f][0], "solve_s": round(tot[f][1], 4),
                                  "value": tot[f][0] / tot[f][1]} for f in forms if tot[f][0]},
        "full_over_split_time": d_full[1] / d_paper[1],
        "roofline": {"kernel": f"additive apply_P, full vertex stars ({big['space']}{big['p']}): patch and coarse "
                               "inverse streams", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None, "bytes_per_launch": nbytes,
                     "launch_us": t_add * 1e6},
        "per_problem": rows,
    }
    print(json.dumps(line), flush=True)


def _timed_solve(prob, b, x, steps, warmup=1):
    import torch
    for _ in range(warmup):
        x.zero_()
        prob.solve(b, x, rtol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        info = prob.solve(b, x, rtol=1e-10)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, info


def mixed_leg(args):
    """Compact mixed-precision comparison for the default line: H(curl) Ned_6
    on the jittered 16^3x6 mesh (mesh seed 4, load seed 5), plain FP64 PCG
    against FP32 refinement and the bfloat16-stored preconditioner, each to
    a true FP64 relative residual of 1e-10 (checked with the FP64 operator)."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    X, C = kuhn_mesh(16, 3, jitter=0.1, seed=4)
    hierarchy = [kuhn_mesh(m, 3) for m in (16, 8, 4, 2, 1)]
    out, ref = {}, None
    for mode in ("fp64", "fp32-ir", "bf16-pc", "fp64+mg", "bf16-pc+mg"):
        prec, _, coarse = mode.partition("+")
        prob = rz.Problem(X, C, 6, "Ned", pc=args.pc, precision=prec, coarse=coarse or "exact",
                          mg_meshes=hierarchy if coarse else None)
        b = torch.from_numpy(load_vectors(prob.n_dofs, 5)[:, 0]).cuda()
        x = torch.zeros_like(b)
        dt, info = _timed_solve(prob, b, x, args.leg_steps)
        y = torch.empty_like(b)
        prob.apply_A(x, y)
        res = ((b - y).norm() / b.norm()).item()
        out[mode] = {"ms": dt * 1e3, "value": prob.n_dofs / dt, "iterations": info["iterations"],
                     "outer_iterations": info["outer_iterations"], "true_rel_residual": res,
                     "setup_ms": round(info["setup_ms"], 1)}
        if ref is None:
            ref = x.clone()
        else:
            out[mode]["rel_diff_vs_fp64_solution"] = ((x - ref).norm() / ref.norm()).item()
        print(f"mixed leg {mode}: {dt * 1e3:.1f} ms, {info['iterations']} its, true residual {res:.2e}",
              file=sys.stderr, flush=True)
        prob.close()
        del b, x, y
        torch.cuda.empty_cache()
    ok = [m for m in out if m != "fp64" and out[m]["true_rel_residual"] <= 1.2e-10]
    best = min(ok, key=lambda m: out[m]["ms"]) if ok else "fp64"
    return {"workload": "H(curl) Ned_6 Riesz map, jittered Kuhn 16^3x6 = 24576 tets, 3,181,344 dofs, to a true "
                        "FP64 rel. residual 1e-10; '+mg': the multigrid V-cycle on W^1 over the Kuhn meshes "
                        "16, 8, 4, 2, 1 in place of the dense coarse inverse", "modes": out, "best": best,
            "speedup_vs_fp64": out["fp64"]["ms"] / out[best]["ms"]}


def multirhs_leg(args):
    """Compact multi-RHS comparison for the default line: H(div) RT_5 on the
    jittered 12^3x6 mesh (mesh seed 6), 64 load vectors (seed 7): one
    batched solve of the 64 columns (FP64 and with the bfloat16-stored
    preconditioner) against the 64 columns solved one by one in FP64."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    X, C = kuhn_mesh(12, 3, jitter=0.1, seed=6)
    nr = args.nrhs
    out = {}
    for mode in ("fp64", "bf16-pc"):
        prob = rz.Problem(X, C, 5, "RT", pc=args.pc, precision=mode)
        B = torch.from_numpy(np.ascontiguousarray(load_vectors(prob.n_dofs, 7, n_rhs=nr).T)).cuda().T
        Xs = torch.zeros_like(B)
        dt, infos = _timed_solve(prob, B, Xs, args.leg_steps)
        Y = torch.empty_like(B)
        prob.apply_A(Xs, Y)
        res = float(((B - Y).norm(dim=0) / B.norm(dim=0)).max())
        its = [i["iterations"] for i in infos]
        out[mode] = {"ms": dt * 1e3, "value": prob.n_dofs * nr / dt, "iterations": {"min": min(its), "max": max(its)},
                     "max_true_rel_residual": res}
        print(f"multi-RHS leg {mode}: {dt * 1e3:.1f} ms for {nr} columns, true residual <= {res:.2e}",
              file=sys.stderr, flush=True)
        if mode == "fp64":
            xs = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j in range(nr):
                xs.zero_()
                prob.solve(B[:, j].contiguous(), xs, rtol=1e-10)
            torch.cuda.synchronize()
            t_seq = time.perf_counter() - t0
            out["fp64_one_by_one"] = {"ms": t_seq * 1e3, "value": prob.n_dofs * nr / t_seq}
        prob.close()
        del B, Xs, Y
        torch.cuda.empty_cache()
    return {"workload": f"H(div) RT_5 Riesz map, jittered Kuhn 12^3x6 = 10368 tets, 946,080 dofs x {nr} right-hand "
                        "sides, rtol 1e-10", "modes": out,
            "speedup_batched_fp64_vs_one_by_one": out["fp64_one_by_one"]["ms"] / out["fp64"]["ms"],
            "speedup_batched_bf16pc_vs_one_by_one": out["fp64_one_by_one"]["ms"] / out["bf16-pc"]["ms"]}


def hodge_leg(args):
    """Compact Hodge-Laplacian leg for the default line: the three complexes
    at p = 4 on the Fichera-corner Freudenthal mesh with 8 cells per edge
    (2688 tets, jitter 0.1 h, mesh seed 31), gamma = 1, split decompositions,
    load uniform[-1, 1] on the X^k equation (seed 32), preconditioned MINRES
    to 1e-8; the true residual by the library's operator apply."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import fichera_mesh
    X, C = fichera_mesh(8, jitter=0.1, seed=31)
    out, tot_dofs, tot_s = {}, 0, 0.0
    for k, name in ((1, "CG4 x Ned4"), (2, "Ned4 x RT4"), (3, "RT4 x DG3")):
        H = rz.Hodge(X, C, 4, k, gamma=1.0)
        b = torch.zeros(H.n, dtype=torch.float64, device="cuda")
        b[H.n0:] = torch.from_numpy(np.random.default_rng(32).uniform(-1, 1, H.n1)).cuda()
        x = torch.empty_like(b)
        H.solve(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.leg_steps):
            info = H.solve(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.leg_steps
        y = torch.empty_like(b)
        H.apply(x, y)
        res = ((b - y).norm() / b.norm()).item()
        out[name] = {"dofs": H.n, "ms": dt * 1e3, "iterations": info["iterations"], "true_rel_residual": res}
        tot_dofs += H.n
        tot_s += dt
        print(f"Hodge leg {name}: {H.n} dofs, {info['iterations']} its, {dt * 1e3:.1f} ms, true residual {res:.1e}",
              file=sys.stderr, flush=True)
        H.close()
        del b, x, y
        torch.cuda.empty_cache()
    return {"workload": "Hodge Laplacians CG_4 x Ned_4, Ned_4 x RT_4, RT_4 x DG_3 on the Fichera-corner Freudenthal "
                        "mesh, 8 cells per edge (2688 tets), gamma = 1, MINRES to 1e-8", "value": tot_dofs / tot_s,
            "unit": "DOF/s", "cases": out}


def spaces_leg(args):
    """Compact leg of the spaces beyond the 3D first kind for the default
    line: 2D Ned_6 and RT_6 on the jittered Kuhn 96^2x2 mesh (mesh seed 2)
    with the W^1 V-cycle over the Kuhn meshes 96, 48, .., 3, and NedTwo_4
    and BDM_4 on the jittered Kuhn 8^3x6 mesh; load seed 3, FP64 PCG to
    1e-10, the default hybrid preconditioner."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    out, tot_dofs, tot_s = {}, 0, 0.0
    X2, C2 = kuhn_mesh(96, 2, jitter=0.1, seed=2)
    h2 = [kuhn_mesh(m, 2) for m in (96, 48, 24, 12, 6, 3)]
    X3, C3 = kuhn_mesh(8, 3, jitter=0.1, seed=2)
    for name, X, C, fam, p, mg in (("2D Ned6 +mg", X2, C2, "Ned", 6, h2), ("2D RT6 +mg", X2, C2, "RT", 6, h2),
                                   ("NedTwo4", X3, C3, "NedTwo", 4, None), ("BDM4", X3, C3, "BDM", 4, None)):
        prob = rz.Problem(X, C, p, fam, pc=args.pc, coarse="mg" if mg else "exact", mg_meshes=mg)
        b = torch.from_numpy(load_vectors(prob.n_dofs, 3)[:, 0]).cuda()
        x = torch.zeros_like(b)
        dt, info = _timed_solve(prob, b, x, args.leg_steps)
        out[name] = {"dofs": prob.n_dofs, "ms": dt * 1e3, "iterations": info["iterations"],
                     "rel_residual": info["rel_residual"], "setup_ms": round(info["setup_ms"], 1)}
        tot_dofs += prob.n_dofs
        tot_s += dt
        print(f"spaces leg {name}: {prob.n_dofs} dofs, {info['iterations']} its, {dt * 1e3:.1f} ms",
              file=sys.stderr, flush=True)
        prob.close()
        del b, x
        torch.cuda.empty_cache()
    return {"workload": "2D Ned_6 / RT_6 (jittered Kuhn 96^2x2, W^1 V-cycle) and NedTwo_4 / BDM_4 (jittered Kuhn "
                        "8^3x6), FP64 PCG to 1e-10", "value": tot_dofs / tot_s, "unit": "DOF/s", "cases": out}


def cpu_baseline(pc="hybrid"):
    """The oracle, as it stands, on a bounded sample of the workload: the
    p = 3 and p = 4 problems of all three spaces of the sweep (same mesh and
    load vectors); CPU DOF/s = dofs / PCG time, setup excluded."""
    from threadpoolctl import threadpool_limits
    from oracle.element import element
    from oracle.mesh import Topology
    from oracle.operator import all_cell_matrices, assemble
    from oracle.pcg import pcg
    from oracle.precond import AdditiveSchwarz, HybridSchwarz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    X, C = kuhn_mesh(8, 3, jitter=0.1, seed=2)
    dofs, t = 0, 0.0
    for fam, p in (("CG", 3), ("CG", 4), ("Ned", 3), ("Ned", 4), ("RT", 3), ("RT", 4)):
        top = Topology(X, C, element(3, fam, p))
        A = assemble(top, all_cell_matrices(top.el, top))
        P = HybridSchwarz(A, top, fam) if pc == "hybrid" else AdditiveSchwarz(A, top, fam)
        b = load_vectors(top.n_dofs, 3)[:, 0]
        with threadpool_limits(1):
            t0 = time.perf_counter()
            _, info = pcg(lambda v: A @ v, P.apply, b, rtol=1e-10)
            t += time.perf_counter() - t0
        dofs += top.n_dofs
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": dofs / t, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"oracle PCG with the {pc} preconditioner (NumPy/SciPy FP64, assembled CSR SpMV, dense "
                      "Cholesky patch solves, BLAS limited to 1 thread) on the p=3 and p=4 problems of H(grad), "
                      f"H(curl) and H(div) of the same sweep ({dofs:,} dofs); setup excluded",
            "seconds": t}


def spaces_workload(args):
    """The solve spaces beyond the 3D first kind: 2D H(curl) Ned_p and 2D
    H(div) RT_p (k = 1, the quarter turn of Ned_p) on the Kuhn mesh of the
    unit square with 96 cells per edge (18,432 triangles, interior vertices
    jittered by 0.1 h, mesh seed 2), p = 2, 4, 6, 8, and the second-kind 3D
    NedTwo_p and BDM_p on the sweep's jittered 8^3x6 mesh, p = 2, 3, 4, 5;
    load seed 3, FP64 PCG to 1e-10 with the hybrid preconditioner of each
    space's default decomposition.  Per case: dofs, setup, iterations (flat in
    p is the paper's robustness claim), solve time and DOF/s.  The 2D cases
    run twice: with the exact coarse solve (in the value) and with the W^1
    V-cycle over the Kuhn meshes 96, 48, 24, 12, 6, 3 (reported beside)."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors
    torch.cuda.set_device(0)
    cases = [("2D", 2, 96, f, p, c) for f in ("Ned", "RT") for p in (2, 4, 6, 8) for c in ("exact", "mg")] + \
            [("3D", 3, args.n, f, p, "exact") for f in ("NedTwo", "BDM") for p in (2, 3, 4, 5)]
    meshes, rows, rows_mg, tot_dofs, tot_s = {}, [], [], 0, 0.0

    def hierarchy(n, d):
        out = [kuhn_mesh(n, d)]
        while n % 2 == 0 and n > 1:
            n //= 2
            out.append(kuhn_mesh(n, d))
        return out

    for label, d, n, fam, p, coarse in cases:
        if (d, n) not in meshes:
            meshes[(d, n)] = kuhn_mesh(n, d, jitter=0.1, seed=2)
        X, C = meshes[(d, n)]
        t0 = time.perf_counter()
        prob = rz.Problem(X, C, p, fam, pc=args.pc, coarse=coarse,
                          mg_meshes=hierarchy(n, d) if coarse == "mg" else None)
        torch.cuda.synchronize()
        t_set = time.perf_counter() - t0
        b = torch.from_numpy(load_vectors(prob.n_dofs, 3)[:, 0]).cuda()
        x = torch.zeros_like(b)
        for _ in range(args.warmup):
            x.zero_()
            prob.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            info = prob.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        (rows if coarse == "exact" else rows_mg).append(
            dict(mesh=label, space=fam, p=p, coarse=coarse, dofs=prob.n_dofs, its=info["iterations"],
                 rel_res=info["rel_residual"], solve_ms=round(dt * 1e3, 3), setup_s=round(t_set, 2),
                 dofs_per_s=prob.n_dofs / dt))
        if coarse == "exact":
            tot_dofs += prob.n_dofs
            tot_s += dt
        print(f"{label} {fam}{p}{' +mg' if coarse == 'mg' else ''}: {prob.n_dofs} dofs, setup {t_set:.2f}s, "
              f"{info['iterations']} its, "
              f"{dt * 1e3:.2f} ms, {prob.n_dofs / dt / 1e6:.1f} M DOF/s", file=sys.stderr, flush=True)
        prob.close()
        del prob
        torch.cuda.empty_cache()
    line = {"metric": "Riesz-map solve DOFs/s to rel. residual 1e-10 (2D and second-kind spaces)",
            "value": tot_dofs / tot_s, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": tot_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"2D Ned_p / RT_p x p = 2,4,6,8 on the jittered Kuhn 96^2x2 mesh and 3D NedTwo_p "
                                   f"/ BDM_p x p = 2..5 on the jittered Kuhn {args.n}^3x6 mesh, rtol 1e-10, "
                                   f"{args.pc} preconditioner; exact coarse solve in the value, the 2D cases "
                                   f"with the W^1 V-cycle beside", "preconditioner": args.pc},
            "cases": rows, "cases_2d_vcycle": rows_mg}
    print(json.dumps(line), flush=True)


def hodge(args):
    """Hodge Laplacians (Sec. 7.2, eq:hodge-laplace) on the Freudenthal mesh
    of the Fichera corner (0,1)^3 minus [1/2,1)^3 with 8 cells per edge
    (2688 tets, interior vertices jittered by 0.1 h, mesh seed 31), load
    uniform[-1, 1] on the X^k equation (seed 32): CG_p x Ned_p,
    Ned_p x RT_p and RT_p x DG_{p-1}, p = 1, 4, 6, gamma = 1 and 1e3, the
    split (paper) and full decompositions, preconditioned MINRES to 1e-8
    (the paper's tolerance) from x = 0; per case setup, iterations, time
    and the true residual ||b - A x|| / ||b|| by the library's own operator
    apply."""
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import fichera_mesh
    torch.cuda.set_device(0)
    X, C = fichera_mesh(8, jitter=0.1, seed=31)
    rows, tot_dofs, tot_s = [], 0, 0.0
    for k, name in ((1, "CG x Ned"), (2, "Ned x RT"), (3, "RT x DG")):
        for p in (1, 4, 6):
            for dec in ("paper", "paper-full"):
                for gamma in (1.0, 1e3):
                    t0 = time.perf_counter()
                    H = rz.Hodge(X, C, p, k, gamma=gamma, decomposition=dec)
                    torch.cuda.synchronize()
                    t_set = time.perf_counter() - t0
                    b = torch.zeros(H.n, dtype=torch.float64, device="cuda")
                    b[H.n0:] = torch.from_numpy(np.random.default_rng(32).uniform(-1, 1, H.n1)).cuda()
                    x = torch.empty_like(b)
                    for _ in range(args.warmup):
                        H.solve(b, x, rtol=1e-8)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(args.steps):
                        info = H.solve(b, x, rtol=1e-8)
                    torch.cuda.synchronize()
                    dt = (time.perf_counter() - t0) / args.steps
                    y = torch.empty_like(b)
                    H.apply(x, y)
                    res = ((b - y).norm() / b.norm()).item()
                    rows.append(dict(complex=name, p=p, decomposition=dec, gamma=gamma, dofs=H.n,
                                     iterations=info["iterations"], ms=round(dt * 1e3, 2), setup_s=round(t_set, 2),
                                     true_rel_residual=res))
                    if dec == "paper":
                        tot_dofs += H.n
                        tot_s += dt
                    print(f"{name} p={p} {dec} gamma={gamma:g}: {H.n} dofs, {info['iterations']} its, "
                          f"{dt * 1e3:.1f} ms, true residual {res:.1e}", file=sys.stderr, flush=True)
                    H.close()
                    torch.cuda.empty_cache()
    line = {"metric": "Hodge-Laplacian MINRES solve DOFs/s to rel. residual 1e-8", "value": tot_dofs / tot_s,
            "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tot_s * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Hodge Laplacians CG_p x Ned_p, Ned_p x RT_p and RT_p x DG_{p-1}, p = 1, 4, 6, "
                                   "gamma = 1 and 1e3, "
                                   "Fichera-corner Freudenthal mesh 8 cells per edge (2688 tets), split "
                                   "decompositions in the value, full ones reported beside them"},
            "cases": rows}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU only; sharding across GPUs is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "multirhs":
        return multirhs(args)
    if args.workload == "mixed":
        return mixed(args)
    if args.workload == "batch":
        return batch_workload(args)
    if args.workload == "hodge":
        return hodge(args)
    if args.workload == "spaces":
        return spaces_workload(args)
    if args.workload == "decompositions":
        return decompositions(args)
    import torch
    from paper_2506_17406_amd import rz
    from paper_2506_17406_amd.workloads import kuhn_mesh, load_vectors

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    X, C = kuhn_mesh(args.n, 3, jitter=0.1, seed=2)
    spaces = args.spaces.split(",")
    degrees = [int(p) for p in args.degrees.split(",")]
    probs = []
    t_setup = time.perf_counter()
    for fam in spaces:
        for p in degrees:
            t0 = time.perf_counter()
            prob = rz.Problem(X, C, p, fam, pc=args.pc)
            b = torch.from_numpy(load_vectors(prob.n_dofs, 3)[:, 0]).cuda()
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            probs.append(dict(fam=fam, p=p, prob=prob, b=b, x=x, setup_s=time.perf_counter() - t0))
            print(f"setup {fam}{p}: {prob.n_dofs} dofs in {probs[-1]['setup_s']:.2f}s", file=sys.stderr, flush=True)
    t_setup = time.perf_counter() - t_setup
    total_dofs = sum(e["prob"].n_dofs for e in probs)

    batch = rz.Batch([e["prob"] for e in probs])

    def step(batched):
        for e in probs:
            e["x"].zero_()
        if batched:
            return batch.solve([e["b"] for e in probs], [e["x"] for e in probs], rtol=1e-10)
        return [e["prob"].solve(e["b"], e["x"], rtol=1e-10) for e in probs]

    def timed(batched):
        for _ in range(args.warmup):
            step(batched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            infos = step(batched)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, infos

    # the headline mode last, so that its solutions are the ones reported
    other = args.sweep_mode != "batched"
    dt_other, infos_other = timed(other)
    dt, infos = timed(not other)
    print(f"timed {args.steps} steps: {dt * 1e3:.1f} ms/step ({args.sweep_mode}); other mode "
          f"{dt_other * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    # operator apply on the largest-flop problem, HIP events on the launch stream
    big = max(probs, key=lambda e: e["prob"].Q * e["prob"].n_loc ** 2)
    pb = big["prob"]
    xa = torch.rand(pb.n_dofs, dtype=torch.float64, device="cuda")
    ya = torch.empty_like(xa)
    for _ in range(3):
        pb.apply_A(xa, ya)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.apply_reps):
        pb.apply_A(xa, ya)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_apply = ev0.elapsed_time(ev1) / 1e3 / args.apply_reps
    flops = 2.0 * pb.Q * pb.n_loc ** 2 * pb.n_cells
    tflops = flops / t_apply / 1e12
    # preconditioner apply on the same problem (HBM-bound stream of packed inverses)
    ev0.record(stream)
    for _ in range(args.apply_reps):
        pb.apply_P(xa, ya)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_prec = ev0.elapsed_time(ev1) / 1e3 / args.apply_reps

    # the preconditioner's largest patch stream: one pass of the family with
    # the most stored inverse bytes, timed on the launch stream
    fam_best = max(((e, k, info) for e in probs for k, info in enumerate(e["prob"].patch_sets())),
                   key=lambda t: t[2]["stored_entries"])
    pe, pk, pinfo = fam_best
    xr = torch.rand(pe["prob"].n_dofs, dtype=torch.float64, device="cuda")
    zr = torch.zeros_like(xr)
    t_patch = _apply_time(lambda u, v: pe["prob"].patch_set_apply(pk, u, v), xr, zr, args.apply_reps, stream)
    # algorithmic bytes: the packed upper triangles (8 bytes per entry), the
    # gathered right-hand side and the read-modify-write of z per patch dof
    patch_bytes = 8.0 * pinfo["packed_entries"] + 24.0 * pinfo["sum_size"]
    fam_names = {("CG", 0): "vertex stars", ("Ned", 0): "edge stars", ("Ned", 1): "vertex-star potentials",
                 ("RT", 0): "edge stars"}
    # HBM traffic of that pass from committed counter runs of the same
    # kernel source (the 855-dof star streams of the n = 8 sweep), else null
    from paper_2506_17406_amd.profile_summary import read_traffic
    trp = read_traffic(os.path.join(ROOT, "profiles", "patch_fold_CG8_sweep_traffic.md"))
    traffic_patch = (float(trp["traffic_bytes_per_launch"])
                     if trp and pe["fam"] == "CG" and pe["p"] == 8 and args.n == 8 else None)
    roofline_patch = {
        "kernel": f"patch solves ({pe['fam']}{pe['p']} {fam_names.get((pe['fam'], pk), 'family %d' % pk)}, "
                  f"{pinfo['n_patches']} patches of <= {pinfo['max_size']} dofs): one pass",
        "bound": "hbm", "achieved": patch_bytes / t_patch / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": patch_bytes / t_patch / 1e9 / PEAK_HBM_GBS, "traffic": traffic_patch, "bytes_per_launch": patch_bytes,
        "stored_bytes": 8.0 * pinfo["stored_entries"], "launch_us": t_patch * 1e6}
    legs = {}
    if not args.no_legs:
        legs["mixed_precision"] = mixed_leg(args)
        legs["multi_rhs"] = multirhs_leg(args)
        legs["hodge"] = hodge_leg(args)
        legs["spaces"] = spaces_leg(args)

    # HBM traffic of the roofline kernel from committed counter runs, if they
    # were taken on the current kernel source
    from paper_2506_17406_amd.profile_summary import read_traffic
    tr = read_traffic(os.path.join(ROOT, "profiles", "apply_A_Ned8_sweep_traffic.md"))
    traffic = float(tr["traffic_bytes_per_launch"]) if tr and big["fam"] == "Ned" and big["p"] == 8 else None
    per = [dict(space=e["fam"], p=e["p"], dofs=e["prob"].n_dofs, its=i["iterations"],
                rel_res=i["rel_residual"], cond=round(i["cond_estimate"], 3), solve_ms=round(i["solve_ms"], 3),
                setup_ms=round(i["setup_ms"], 1), cells_per_wave=e["prob"].apply_tiles())
           for e, i in zip(probs, infos)]
    line = {
        "metric": "Riesz-map solve DOFs/s to rel. residual 1e-10",
        "value": total_dofs / dt,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D plain FP64 PCG sweep: H(grad)/H(curl)/H(div) x p={args.degrees} on the "
                               f"jittered Kuhn mesh {args.n}^3x6 = {6 * args.n ** 3} tets, rtol 1e-10",
                   "problems": len(probs), "total_dofs": total_dofs, "setup_s": round(t_setup, 2),
                   "preconditioner": args.pc, "mode": args.sweep_mode},
        "roofline": {"kernel": f"apply_A ({big['fam']}{big['p']}): cell gather, GEMM, assembly",
                     "bound": "mfma",
                     "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops, "launch_us": t_apply * 1e6},
        "roofline_patch": roofline_patch,
        "apply_P_us": t_prec * 1e6,
        ("sequential" if args.sweep_mode == "batched" else "batched"): {
            "value": total_dofs / dt_other, "ms_per_step": dt_other * 1e3,
            "iterations": [i["iterations"] for i in infos_other]},
        "per_problem": per,
    }
    line.update(legs)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.pc)
    print(json.dumps(line), flush=True)
    if args.profile_copy_bytes > 0:
        src = torch.empty(args.profile_copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
