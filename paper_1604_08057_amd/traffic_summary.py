"""Turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) of ``bench.py --copy-probe``
into the per-dispatch HBM traffic summary that bench.py reads.

Each counter is scaled by what it reads for the probe's three 1 GiB device copies
(the first three dispatches of each run).  Usage:
    python -m paper_1604_08057_amd.traffic_summary FETCH.csv WRITE.csv OUT.txt
"""
from __future__ import annotations

import csv
import hashlib
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


def site_workgroups(dims) -> int:
    """Workgroups per source of the colour-split kernels: the library's site-block
    order (segments of every t-slice per XCD when a segment's stencil-pair data fits
    in half an XCD's L2, else contiguous runs), lists padded to equal length."""
    nx, ny, nz, nt = dims
    V, V3 = nx * ny * nz * nt, nx * ny * nz
    nsb = ((V + 63) // 64 + 7) // 8 * 8
    if V3 / 8 * 1728 > 2 * 1024 * 1024:
        return nsb
    per = [0] * 8
    for b in range(nsb):
        per[((b * 64) % V3) * 8 // V3] += 1
    return max(per) * 8


def main(fetch_csv: str, write_csv: str, out: str, volume: int = 4096):
    F = list(csv.DictReader(open(fetch_csv)))
    W = list(csv.DictReader(open(write_csv)))
    probe = [(a, b) for a, b in zip(F, W) if "copyBuffer" in a["Kernel_Name"]][:3]
    cf = statistics.mean(float(a["Counter_Value"]) for a, _ in probe)
    cw = statistics.mean(float(b["Counter_Value"]) for _, b in probe)
    ff, fw = PROBE_BYTES / 1024 / cf, PROBE_BYTES / 1024 / cw

    def sel(name, grid=None):
        return [(a, b) for a, b in zip(F, W) if a["Kernel_Name"].startswith(f"void tslov::{name}(")
                and (grid is None or a["Grid_Size"] == grid)]

    def per(name, grid):
        s = sel(name, grid)
        return (len(s), statistics.mean(float(a["Counter_Value"]) for a, _ in s),
                statistics.mean(float(b["Counter_Value"]) for _, b in s))

    V = volume
    ncol = 3 * (((V + 63) // 64 + 7) // 8 * 8) * 64    # colour-grid threads at this volume
    npt = (V + 255) // 256 * 256 * 12                  # pointwise kernels
    rows = {"k_fwd_pair<double>": (str(3 * ncol), V * (6 * 12 + 36) * 16),
            "k_bwd_rb_cg<double>": (str(3 * ncol), V * (12 * 12 + 36) * 16),
            "k_recur<double>": (str(npt), V * 8 * 12 * 16),
            "k_bwd_ra<double>": (str(npt), V * 10 * 12 * 16)}
    lines = ["# HBM traffic per dispatch from rocprofv3 counters, 8^4 workload (V=4096, k=200, FP64)",
             "#",
             "# commands (repository root on the GPU box as $REPO), one counter per pass:",
             "#   cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \\",
             "#     \"k_fwd_pair|k_bwd_rb|k_apply|copy|k_recur|k_bwd_ra|k_force\" -f csv -d $REPO/gpurun_out/pmc_fetch"
             " -o run -- \\",
             "#     python3 $REPO/bench.py --steps 2 --warmup 1 --no-cpu-baseline --copy-probe",
             "#   (the same with --pmc WRITE_SIZE into $REPO/gpurun_out/pmc_write), then",
             "#   python -m paper_1604_08057_amd.traffic_summary pmc_fetch/run_counter_collection.csv \\",
             "#     pmc_write/run_counter_collection.csv profiles/traffic_stencil_pair_8x8x8x8.txt",
             "#",
             f"# calibration: the probe's three 1 GiB device copies read FETCH_SIZE {cf:.1f} KiB and",
             f"#   WRITE_SIZE {cw:.1f} KiB per dispatch: scale factors fetch x{ff:.4f}, write x{fw:.4f}",
             "#",
             "# kernel                          grid   dispatches  FETCH_KiB  WRITE_KiB  hbm_bytes(scaled)  algorithmic"]
    res = {}
    for name, (grid, alg) in rows.items():
        n, f, w = per(name, grid)
        res[name] = (f * ff + w * fw) * 1024
        lines.append(f"{name:31s} {grid:>7s} {n:10d} {f:10.1f} {w:10.1f} {res[name]:18.0f} {alg:12d}")
    # the 32^4 operator of the stencil benchmark (t-march: 256 tiles x 2 chunks of 16 slices)
    V4 = 32 ** 4
    g4 = str(32 ** 3 // 128 * 2 * 128)
    try:
        n, f, w = per("k_apply_tmarch<double>", g4)
        lines.append(f"{'k_apply_tmarch<double> (32^4)':31s} {g4:>7s} {n:10d} {f:10.1f} {w:10.1f} "
                     f"{(f * ff + w * fw) * 1024:18.0f} {V4 * 60 * 16:12d}")
    except statistics.StatisticsError:
        pass
    # the batched 6x18^3 workload's FP64 stencil pairs (colour split, one entry per
    # workgroup as the tuner picks, sources in memory-sized groups): every dispatch
    # on this lattice, per entry-step; algorithmic = the entry's fields + the links
    # once per launch, spread over the launch's entries
    Vb, per_src = 6 * 18 ** 3, site_workgroups((18, 18, 18, 6)) * 192
    for base, planes in (("k_fwd_pair_ms", 6 * 12), ("k_bwd_rb_ms", 12 * 12)):
        name = f"{base}<double, 1>"
        s_ = [(a, b) for a, b in sel(name) if int(a["Grid_Size"]) % per_src == 0]   # this lattice only
        entries = sum(int(a["Grid_Size"]) // per_src for a, _ in s_)
        if entries:
            f = sum(float(a["Counter_Value"]) for a, _ in s_) / entries
            w = sum(float(b["Counter_Value"]) for _, b in s_) / entries
            alg = Vb * planes * 16 + Vb * 36 * 16 * len(s_) // entries
            lines.append(f"{name + ' (6x18^3)':31s} {'/entry':>7s} {len(s_):10d} {f:10.1f} {w:10.1f} "
                         f"{(f * ff + w * fw) * 1024:18.0f} {alg:12d}")
    lines += ["#", "# read by bench.py (the stencil pair kernels of the timed 8^4 step):",
              "kernel: k_bwd_rb_cg<double>",
              f"hbm_bytes_per_launch: {res['k_bwd_rb_cg<double>']:.0f}",
              f"fwd_pair_hbm_bytes_per_launch: {res['k_fwd_pair<double>']:.0f}",
              f"kernel_source_sha256_16: {kernel_source_hash()}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main(*sys.argv[1:4])
