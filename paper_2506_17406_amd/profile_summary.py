"""Summaries of rocprofv3 output for the profiles directory.

    python -m paper_2506_17406_amd.profile_summary stats <results.db> [top]
        per-kernel calls and durations of a --kernel-trace --stats run
        (rocpd SQLite) as a Markdown table;
    python -m paper_2506_17406_amd.profile_summary traffic <fetch.csv> <write.csv> <kernel> <copy_bytes> [grid]
        HBM bytes per operator apply whose GEMM is <kernel> (with the gather
        and assembly dispatched around it; with grid, only GEMM dispatches of
        that many work-items, i.e. one problem's applies) from two --pmc runs
        (FETCH_SIZE, then WRITE_SIZE; counter_collection CSVs), each scaled by
        what the same counter reads for the plain copy kernel of copy_bytes
        bytes read and written in the same run.  Prints key: value lines;
    python -m paper_2506_17406_amd.profile_summary mfma <counters.csv> <kernel> [grid]
        MFMA use of <kernel> (of grid work-items if given) from a --pmc run of
        SQ_VALU_MFMA_BUSY_CYCLES and SQ_INSTS_VALU_MFMA_MOPS_F64: the FP64
        MFMA flops counted (512 per MOP) over each dispatch's own duration
        (its start/end timestamps) against the 78.6 TFLOP/s FP64 peak, and
        the busy cycles over duration x 2.4 GHz x 1024 SIMDs;
    python -m paper_2506_17406_amd.profile_summary bandwidth <fetch.csv> <write.csv> <results.db> <copy_bytes> [top]
        per kernel name: mean HBM bytes per dispatch (counters scaled by the
        copy kernel, as for traffic) over mean duration in a kernel trace;
    python -m paper_2506_17406_amd.profile_summary kernel_traffic <fetch.csv> <write.csv> <kernel> <copy_bytes> [grid|max]
        HBM bytes per dispatch of one kernel (of that grid, or its largest
        grid), scaled by the copy kernel as for traffic; key: value lines;
    python -m paper_2506_17406_amd.profile_summary applies <results.db> <kernel> [grid_y]
        mean duration of those applies (gather start to assembly end) and of
        their GEMM kernel in a kernel trace (with grid_y, only GEMM dispatches
        of that many row blocks).
"""
import collections
import csv
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def short(name):
    name = name.replace("rz::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def summarise(db, top=30):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = ["| kernel | calls | total (us) | average (us) | % of GPU time |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows[:top]:
        out.append(f"| {short(name)} | {calls} | {tot:.1f} | {avg:.2f} | {pct:.2f} |")
    return "\n".join(out)


def kernels_sha256():
    """Hash of the device kernel source; a traffic figure is only valid for it."""
    with open(os.path.join(HERE, "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


# one operator apply = cell gather, the GEMM kernel, assembly (base names,
# template arguments dropped)
APPLY_PARTS = ("k_gather_cells", "GEMM", "k_assemble")


def base(name):
    return name.split("<")[0]


def _dispatches(path, counter):
    """(dispatch id, short kernel name, value, grid work-items) in dispatch order."""
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), short(r["Kernel_Name"]), float(r["Counter_Value"]),
                        int(r["Grid_Size"])))
    return sorted(out)


def _apply_sums(rows, kernel, grid=None):
    """Counter sums over each operator apply whose GEMM is `kernel` (of
    `grid` work-items if given): the gather dispatched just before it and the
    assembly just after."""
    sums = []
    for i, (_, name, v, g) in enumerate(rows):
        if name != kernel or i < 1 or i + 1 >= len(rows) or (grid and g != grid):
            continue
        if base(rows[i - 1][1]) == APPLY_PARTS[0] and base(rows[i + 1][1]) == APPLY_PARTS[2]:
            sums.append(rows[i - 1][2] + v + rows[i + 1][2])
    return sums


def traffic(fetch_csv, write_csv, kernel, copy_bytes, grid=None):
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")

    def copy_kib(rows):
        # the copy kernel: the dispatch whose counter is closest to copy_bytes
        cands = [v for _, name, v, _ in rows if "copy" in name.lower() or "elementwise" in name.lower()]
        return min(cands, key=lambda v: abs(v * 1024 - copy_bytes))

    ff = copy_bytes / (copy_kib(f) * 1024)
    fw = copy_bytes / (copy_kib(w) * 1024)
    fs, ws = _apply_sums(f, kernel, grid), _apply_sums(w, kernel, grid)
    fk, wk = sum(fs) / len(fs), sum(ws) / len(ws)
    t = fk * 1024 * ff + wk * 1024 * fw
    return {"kernel": kernel + " with its gather and assembly" + (f", GEMM grid {grid}" if grid else ""),
            "kernels_hip_sha256": kernels_sha256(),
            "fetch_kib_per_apply": fk, "write_kib_per_apply": wk, "applies": len(fs), "copy_bytes": copy_bytes,
            "copy_fetch_factor": ff, "copy_write_factor": fw, "traffic_bytes_per_launch": t}


def kernel_traffic(fetch_csv, write_csv, kernel, copy_bytes, grid=None):
    """HBM bytes per dispatch of one kernel (of `grid` work-items; "max": the
    largest grid it ran on) from the two counter runs, scaled by the copy
    kernel's readings as in `traffic`."""
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")

    def copy_kib(rows):
        cands = [v for _, name, v, _ in rows if "copy" in name.lower() or "elementwise" in name.lower()]
        return min(cands, key=lambda v: abs(v * 1024 - copy_bytes))

    if grid == "max":
        grid = max(g for _, name, _, g in f if name == kernel)
    ff = copy_bytes / (copy_kib(f) * 1024)
    fw = copy_bytes / (copy_kib(w) * 1024)
    fs = [v for _, name, v, g in f if name == kernel and (not grid or g == int(grid))]
    ws = [v for _, name, v, g in w if name == kernel and (not grid or g == int(grid))]
    # dispatches that did the work (inside PCG chunks, launches that found
    # their column converged exit at once and read almost nothing)
    fs = [v for v in fs if v >= 0.5 * max(fs)]
    ws = [v for v in ws if v >= 0.5 * max(ws)]
    fk, wk = sum(fs) / len(fs), sum(ws) / len(ws)
    return {"kernel": kernel + (f", grid {grid}" if grid else ""), "kernels_hip_sha256": kernels_sha256(),
            "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": len(fs),
            "copy_bytes": copy_bytes, "copy_fetch_factor": ff, "copy_write_factor": fw,
            "traffic_bytes_per_launch": fk * 1024 * ff + wk * 1024 * fw}


def apply_durations(db, kernel, grid_y=None):
    """Durations (us) of the operator applies whose GEMM is `kernel` (with
    grid_y row blocks if given) in a kernel trace: from the start of the
    gather to the end of the assembly."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, grid_y from kernels order by start").fetchall()
    out = []
    gys = [gy for _, _, _, gy in rows]
    rows = [(short(n), s, e) for n, s, e, _ in rows]
    for i, (name, s, e) in enumerate(rows):
        if name != kernel or i < 1 or i + 1 >= len(rows) or (grid_y and gys[i] != grid_y):
            continue
        if base(rows[i - 1][0]) == APPLY_PARTS[0] and base(rows[i + 1][0]) == APPLY_PARTS[2]:
            out.append(((rows[i + 1][2] - rows[i - 1][1]) / 1e3, (e - s) / 1e3))
    return out


SIMDS = 256 * 4  # MI355X: 256 CUs of 4 SIMDs, 2.4 GHz, FP64 MFMA 78.6 TFLOP/s
CLOCK_HZ = 2.4e9
PEAK_FP64 = 78.6e12


def mfma(path, kernel, grid=None):
    per = collections.defaultdict(dict)
    for r in csv.DictReader(open(path)):
        if short(r["Kernel_Name"]) != kernel or (grid and int(r["Grid_Size"]) != grid):
            continue
        d = per[int(r["Dispatch_Id"])]
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    # dispatches that did work (launches that found their column converged exit at once)
    rows = [d for d in per.values() if d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0) > 0 and d["ns"] > 10e3]
    flops = sum(d["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512 for d in rows) / len(rows)
    ns = sum(d["ns"] for d in rows) / len(rows)
    busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) / (d["ns"] * 1e-9 * CLOCK_HZ * SIMDS) for d in rows) / len(rows)
    return {"kernel": kernel + (f", grid {grid}" if grid else ""), "dispatches": len(rows),
            "fp64_mfma_flops_per_dispatch": flops, "mean_duration_us": ns / 1e3,
            "fp64_mfma_tflops": flops / (ns * 1e-9) / 1e12, "fraction_of_fp64_peak": flops / (ns * 1e-9) / PEAK_FP64,
            "mfma_busy_cycles_fraction": busy}


def bandwidth(fetch_csv, write_csv, db, copy_bytes, top=20):
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")

    def copy_kib(rows):
        cands = [v for _, name, v, _ in rows if "copy" in name.lower() or "elementwise" in name.lower()]
        return min(cands, key=lambda v: abs(v * 1024 - copy_bytes))

    ff, fw = copy_bytes / (copy_kib(f) * 1024), copy_bytes / (copy_kib(w) * 1024)
    by = collections.defaultdict(lambda: [0.0, 0])
    for rows, fac in ((f, ff), (w, fw)):
        for _, name, v, _ in rows:
            by[name][0] += v * 1024 * fac
    for _, name, _, _ in f:
        by[name][1] += 1
    con = sqlite3.connect(db)
    dur = collections.defaultdict(list)
    for n, d in con.execute("select name, duration from kernels").fetchall():
        dur[short(n)].append(d)
    out = ["| kernel | dispatches (counters) | mean MB per dispatch | mean duration (us) | GB/s |",
           "|---|---|---|---|---|"]
    rows = []
    for name, (b, n) in by.items():
        ds = [d for d in dur.get(name, []) if d > 0]
        if not ds or n == 0:
            continue
        mb = b / n / 1e6
        us = sum(ds) / len(ds) / 1e3
        rows.append((b / n / (us * 1e-6) / 1e9 * (us > 0), name, n, mb, us))
    tot = {name: sum(dur.get(name, [0])) for name in by}
    for gbs, name, n, mb, us in sorted(rows, key=lambda r: -tot[r[1]])[:top]:
        out.append(f"| {name} | {n} | {mb:.2f} | {us:.1f} | {gbs:.0f} |")
    return "\n".join(out)


def read_traffic(path):
    """key: value lines written by `traffic`, or None if the file is missing
    or the kernel source has changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    d = {}
    for line in open(path):
        m = re.match(r"^([a-z_0-9]+): (.+)$", line.strip())
        if m:
            d[m.group(1)] = m.group(2)
    if d.get("kernels_hip_sha256") != kernels_sha256():
        return None
    return d


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(summarise(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 30))
    elif sys.argv[1] == "traffic":
        grid = int(sys.argv[6]) if len(sys.argv) > 6 else None
        for k, v in traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), grid).items():
            print(f"{k}: {v}")
    elif sys.argv[1] == "mfma":
        grid = int(sys.argv[4]) if len(sys.argv) > 4 else None
        for k, v in mfma(sys.argv[2], sys.argv[3], grid).items():
            print(f"{k}: {v}")
    elif sys.argv[1] == "bandwidth":
        print(bandwidth(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]),
                        int(sys.argv[6]) if len(sys.argv) > 6 else 20))
    elif sys.argv[1] == "kernel_traffic":
        grid = sys.argv[6] if len(sys.argv) > 6 else None
        for k, v in kernel_traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), grid).items():
            print(f"{k}: {v}")
    elif sys.argv[1] == "applies":
        gy = int(sys.argv[4]) if len(sys.argv) > 4 else None
        d = [a for a in apply_durations(sys.argv[2], sys.argv[3], gy) if a[1] > 10.0]
        print(f"applies: {len(d)}")
        print(f"apply_us_mean: {sum(a[0] for a in d) / len(d):.1f}")
        print(f"gemm_us_mean: {sum(a[1] for a in d) / len(d):.1f}")
