"""Turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) of
``bench.py --copy-probe --no-extras --no-cpu-baseline`` into the per-dispatch HBM
traffic summary that bench.py reads.

Each counter is scaled by what it reads for the probe's three 1 GiB device copies
(the first three dispatches of each run): FETCH_SIZE and WRITE_SIZE count in KiB,
and the copy's known bytes fix their scale.  The batched stencil pair kernels of
the timed call (the class the bench line's ``roofline`` names, e.g. float64
links and vectors; the last dispatches of that class in the run: as many as the
line reports for its timed steps) are
averaged per dispatch, the quantity bench.py sets beside its algorithmic bytes per
launch.  Usage:
    python -m paper_1604_08057_amd.traffic_summary FETCH.csv WRITE.csv BENCH.json OUT.txt
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("common.h", "fields.hip"):
        with open(os.path.join(ROOT, "paper_1604_08057_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _bench_line(path: str) -> dict:
    for line in open(path):
        line = line.strip()
        if line.startswith("{") and '"metric"' in line:
            return json.loads(line)
    raise ValueError(f"no bench JSON line in {path}")


def main(fetch_csv: str, write_csv: str, bench_json: str, out: str):
    F = list(csv.DictReader(open(fetch_csv)))
    W = list(csv.DictReader(open(write_csv)))
    b = _bench_line(bench_json)
    probe = [(x, y) for x, y in zip(F, W) if "copyBuffer" in x["Kernel_Name"]][:3]
    cf = statistics.mean(float(x["Counter_Value"]) for x, _ in probe)
    cw = statistics.mean(float(y["Counter_Value"]) for _, y in probe)
    ff, fw = PROBE_BYTES / 1024 / cf, PROBE_BYTES / 1024 / cw

    def sel(prefix):
        return [(x, y) for x, y in zip(F, W) if x["Kernel_Name"].startswith(f"void tslov::{prefix}")]

    rf = b["roofline"]
    dom_fwd = rf["kernel"].startswith("k_fwd_pair")
    links = ", float>" if ", float>" in rf["kernel"] else ", double>"
    lines = ["# HBM traffic per dispatch from rocprofv3 counters: batched stencil pair kernels of the",
             f"# 6x18^3 batching workload (32 sources, k in [100, 400]; kernel class <double, NS{links})",
             "#",
             "# commands (repository root on the GPU box as $REPO), one counter per pass:",
             "#   cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \\",
             "#     \"k_fwd_pair_ms|k_bwd_rb_ms|copy\" -f csv -d $REPO/gpurun_out/pmc_fetch -o run -- \\",
             "#     python3 $REPO/bench.py --steps 1 --warmup 1 --no-extras --no-cpu-baseline --copy-probe",
             "#   (the same with --pmc WRITE_SIZE into $REPO/gpurun_out/pmc_write, its bench line in",
             "#   $REPO/gpurun_out/pmc_write.json), then",
             "#   python -m paper_1604_08057_amd.traffic_summary pmc_fetch/run_counter_collection.csv \\",
             "#     pmc_write/run_counter_collection.csv pmc_write.json profiles/traffic_batched_pair_6x18x18x18.txt",
             "#",
             f"# calibration: the probe's three 1 GiB device copies read FETCH_SIZE {cf:.1f} KiB and",
             f"#   WRITE_SIZE {cw:.1f} KiB per dispatch: scale factors fetch x{ff:.4f}, write x{fw:.4f}",
             "#",
             "# kernel (timed call's dispatches)            dispatches  FETCH_KiB  WRITE_KiB  hbm_bytes(scaled)  "
             "algorithmic(bench)"]
    res = {}
    for tag, prefix, is_fwd in (("fwd", "k_fwd_pair_ms<double, ", True), ("bwd", "k_bwd_rb_ms<double, ", False)):
        rows = [(x, y) for x, y in sel(prefix) if links in x["Kernel_Name"]]
        src = rf if is_fwd == dom_fwd else rf["other_pair"]
        n_last, alg = int(src["launches"]), float(src["bytes_per_launch"])
        rows = rows[-n_last:]
        if not rows:
            continue
        f = statistics.mean(float(x["Counter_Value"]) for x, _ in rows)
        w = statistics.mean(float(y["Counter_Value"]) for _, y in rows)
        res[tag] = (f * ff + w * fw) * 1024
        name = rows[0][0]["Kernel_Name"].split("(")[0].replace("void tslov::", "")
        a = f"{alg:.0f}" if alg else "-"
        lines.append(f"{name:44s} {len(rows):10d} {f:10.1f} {w:10.1f} {res[tag]:18.0f}  {a}")
    lines += ["#", "# read by bench.py (mean over the timed call's dispatches of each class):",
              f"fwd_pair_hbm_bytes_per_launch: {res.get('fwd', float('nan')):.0f}",
              f"bwd_pair_hbm_bytes_per_launch: {res.get('bwd', float('nan')):.0f}",
              f"kernel_source_sha256_16: {kernel_source_hash()}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main(*sys.argv[1:5])
