"""Per-kernel summary of a rocprofv3 kernel-trace results database (``-o run`` writes
``run_results.db``): calls, total and mean duration, share of kernel time.  Usage:
    python -m paper_1604_08057_amd.kernel_summary RUN_results.db [TOP]
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


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25))
