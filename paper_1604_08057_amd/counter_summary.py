"""Mean counter values per dispatch from rocprofv3 ``--pmc ... -f csv`` runs, for the last
N dispatches of each kernel whose name contains a given text (the timed launches of a
bench run are the last ones of their kernel).  Usage:
    python -m paper_1604_08057_amd.counter_summary TEXT N RUN_counter_collection.csv [...]
"""
from __future__ import annotations

import collections
import csv
import statistics
import sys


def summarise(text: str, last: int, paths) -> str:
    by = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        for r in csv.DictReader(open(path)):
            if text in r["Kernel_Name"]:
                name = r["Kernel_Name"].split("(")[0].replace("void tslov::", "")
                by[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = []
    for name, counters in sorted(by.items()):
        for cname, vals in sorted(counters.items()):
            sel = vals[-last:]
            out.append(f"{name:44s} {cname:32s} {len(sel):6d} {statistics.mean(sel):14.4e}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1], int(sys.argv[2]), sys.argv[3:]))
