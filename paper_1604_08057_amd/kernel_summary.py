"""Per-kernel summary of a rocprofv3 kernel-trace results database (``-o run`` writes
``run_results.db``): calls, total and mean duration, share of kernel time.  Given the
bench.py JSON line of the same run, it also gives the mean duration of exactly the
timed launches of the line's roofline kernels (the last launches of their kernel,
as many as the line counts), the figure to set beside the line's HIP-event mean.
Usage:
    python -m paper_1604_08057_amd.kernel_summary RUN_results.db [TOP] [BENCH_JSON]
"""
from __future__ import annotations

import re
import sqlite3
import sys


def summarise(db_path: str, top: int = 25) -> str:
    db = sqlite3.connect(db_path)
    rows = list(db.execute("select name, count(*), sum(end - start), avg(end - start) from kernels group by name"))
    tot = sum(r[2] for r in rows)
    out = [f"# total kernel time {tot / 1e6:.2f} ms over {sum(r[1] for r in rows)} launches",
           f"# {'kernel':56s} {'calls':>7s} {'total_us':>12s} {'mean_us':>9s} {'pct':>6s}"]
    for name, calls, t, avg in sorted(rows, key=lambda r: -r[2])[:top]:
        short = re.sub(r"\(.*", "", name).replace("tslov::", "").replace("void ", "")
        out.append(f"{short[:58]:58s} {calls:7d} {t / 1e3:12.1f} {avg / 1e3:9.2f} {100 * t / tot:6.2f}")
    return "\n".join(out)


def timed_launches(db_path: str, bench_json: str) -> str:
    import json
    line = next(x for x in open(bench_json) if x.strip().startswith("{") and '"metric"' in x)
    rf = json.loads(line)["roofline"]
    db = sqlite3.connect(db_path)
    out = ["# timed launches of the bench line's roofline kernels (last launches of each kernel):",
           f"# {'kernel':56s} {'launches':>8s} {'trace_mean_us':>14s} {'bench_mean_us':>14s}"]
    for k in (rf, rf["other_pair"]):
        name = re.sub(r" \(.*", "", k["kernel"]).replace("NS", "1")
        n = int(k["launches"])
        rows = list(db.execute("select end - start from kernels where name like ? order by start",
                               (f"%tslov::{name}(%",)))
        sel = [r[0] for r in rows[-n:]]
        mean = sum(sel) / len(sel) / 1e3 if sel else float("nan")
        out.append(f"{name[:58]:58s} {len(sel):8d} {mean:14.2f} {k['mean_us']:14.2f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25))
    if len(sys.argv) > 3:
        print(timed_launches(sys.argv[1], sys.argv[3]))
