"""Summaries of rocprofv3 output for the profiles directory.

    python -m paper_2506_17406_amd.profile_summary stats <results.db> [top]
        per-kernel calls and durations of a --kernel-trace --stats run
        (rocpd SQLite) as a Markdown table;
    python -m paper_2506_17406_amd.profile_summary traffic <fetch.csv> <write.csv> <kernel> <copy_bytes>
        HBM bytes per dispatch of <kernel> from two --pmc runs (FETCH_SIZE,
        then WRITE_SIZE; counter_collection CSVs), each scaled by what the
        same counter reads for the plain copy kernel of copy_bytes bytes
        read and written in the same run.  Prints key: value lines.
"""
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


def _per_dispatch(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv, write_csv, kernel, copy_bytes):
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")

    def copy_kib(vals):
        # the copy kernel: the dispatch whose counter is closest to copy_bytes
        cands = [v for name, vs in vals.items() if "copy" in name.lower() or "elementwise" in name.lower() for v in vs]
        return min(cands, key=lambda v: abs(v * 1024 - copy_bytes))

    ff = copy_bytes / (copy_kib(f) * 1024)
    fw = copy_bytes / (copy_kib(w) * 1024)
    fk = sum(f[kernel]) / len(f[kernel])
    wk = sum(w[kernel]) / len(w[kernel])
    t = fk * 1024 * ff + wk * 1024 * fw
    return {"kernel": kernel, "kernels_hip_sha256": kernels_sha256(), "fetch_kib_per_dispatch": fk,
            "write_kib_per_dispatch": wk, "dispatches": len(f[kernel]), "copy_bytes": copy_bytes,
            "copy_fetch_factor": ff, "copy_write_factor": fw, "traffic_bytes_per_launch": t}


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
        for k, v in traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])).items():
            print(f"{k}: {v}")
