"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as a Markdown
table of per-kernel call counts and durations."""
import re
import sqlite3
import sys


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


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30))
