#!/usr/bin/env python3
"""Benchmark of the TSL sign function + all-links derivative on one MI355X.

One step = one pass of the whole hot path over one batch: the 6x18^3 batching
workload (V = 34992, n = 419904, Wilson mass -2, mu = 0.5, SU(3) link spread
0.35), 32 Z2-complex sources with Krylov sizes drawn uniformly from [100, 400],
each source's sgn(H)psi and its full derivative dS/dU over all 4V links of
S = Re <eta|sgn(H)|psi>, in one tslov_sign_grad_batched call, with every input
resident in HBM.  The headline runs float64 throughout: it is bit-identical to
the single-source path, and it is also the fastest batch that meets 1e-6 on every
output (the float32-link batch is no faster and misses 1e-6 on S and dS/dU at
these Krylov sizes; the float32-vector batch is faster and wrong).  Beside it the
line states the plain float64 single-source path on the same 32 sources (the
comparison the metric names), and the float32-link and float32-vector batches
with their per-output errors against the float64 batch.

The JSON line carries:
* value: sources/s of the batched float64 path over the timed steps;
* roofline: the dominant batched stencil kernel (forward or reverse pair) over
  the timed steps: algorithmic bytes per launch (every entry's fields, the links
  once per launch) over its mean duration from HIP events on the library stream;
  traffic from the committed counter summary when it matches the kernel source;
* cpu_baseline: the CPU oracle (torch/NumPy float64 forward TSL + autograd
  gradient) on a bounded sample of the same workload, scaled to sources/s;
* single_8x8x8x8: the 8^4 workload (k = 200) single source, float64;
* precision_14x14x14x14: the 14^4 workload (k = 400) single source in float64,
  float32 links and float32 vectors, with the per-output errors;
* stencil_large: the float64 Wilson stencil alone on a 32^4 lattice (1.15 GB per
  application, above the 256 MB last-level cache) for the HBM-bound figure.
With --copy-probe a 1 GiB device-to-device copy runs first (HBM counter
calibration for rocprofv3 --pmc).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sgn(H)ψ+dU-derivative sources/s, mixed vs FP64 @≤1e-6 rel; stencil HBM GB/s"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "k_fwd_pair_ms<double, NS, double> (batched fused Lanczos stencil pair, colour split)",
                1: "k_bwd_rb_ms<double, NS, double> (batched reverse-mode stencil pair, colour split)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batched_pair_6x18x18x18.txt")
# live kernel timing samples every 16th launch of the single-source classes: an event
# pair adds ~5 us of dispatch latency, which on every launch would slow a small step
TIMING_EVERY = 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def read_traffic(which: int):
    """HBM bytes per launch of the batched stencil pair kernel (0 forward, 1 reverse)
    from the committed counter summary, or None if absent or taken on a different
    kernel source."""
    from paper_1604_08057_amd.traffic_summary import kernel_source_hash
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["bwd_pair_hbm_bytes_per_launch" if which == 1 else "fwd_pair_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_t(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def batch_errors(S, dU, y, S64, dU64, y64):
    n = len(S)
    e = {"y": max(rel_t(y[s], y64[s]) for s in range(n)),
         "S": max(abs(S[s] - S64[s]) / abs(S64[s]) for s in range(n)),
         "dU": max(rel_t(dU[s], dU64[s]) for s in range(n))}
    dus = sorted(rel_t(dU[s], dU64[s]) for s in range(n))
    e["dU_median"] = dus[n // 2]
    return e


def headline(steps: int, warmup: int):
    """The batched 6x18^3 workload: the float64 batch timed, with the float32-link
    batch, the float64 single-source path and the float32-vector batch beside it."""
    import numpy as np
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(4)
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    ks = [int(k) for k in wl.krylov_sizes()]
    n = len(ks)
    out = {}

    # the float64 batch: the first call allocates and tunes; its results are the
    # reference of the single-source comparison and of the error columns
    ctx = Context(wl.dims, wl.mass, wl.mu, precision="fp64")
    ctx.set_links(U)
    for _ in range(max(warmup, 1)):
        S64, dU64, _, infos, y64 = ctx.sign_grad_batched(eta, psi, ks, want_y=True)
    torch.cuda.synchronize()

    # the plain float64 single-source path on the same 32 sources (before the timed
    # steps, so that the timed launches are the last of their kernels in a trace)
    dU1 = torch.empty_like(dU64[0])
    ctx.sign_grad(eta[0], psi[0], ks[0], dU=dU1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = None
    for s in range(n):
        Ss, _, _, _, ys = ctx.sign_grad(eta[s], psi[s], ks[s], dU=dU1, want_y=True)
        if same is None and ks[s] >= 300:
            torch.cuda.synchronize()
            same = bool(Ss == S64[s] and torch.equal(dU1, dU64[s]) and torch.equal(ys, y64[s]))
    torch.cuda.synchronize()
    out["fp64_single_source_sources_per_s"] = n / (time.perf_counter() - t0)
    out["fp64_batch_identical_to_single_k_ge_300"] = same
    log(f"bench: fp64 single source {out['fp64_single_source_sources_per_s']:.2f} sources/s")
    del dU1

    # the timed path: the float64 batch
    ctx.sign_grad_batched(eta, psi, ks, want_y=True)     # back to the batch's workspace shape
    torch.cuda.synchronize()
    ctx.timing_enable(1)      # batched launches are long: an event pair on each costs < 1%
    ctx.timing_read(0)
    ctx.timing_read(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S64, dU64, _, infos, y64 = ctx.sign_grad_batched(eta, psi, ks, want_y=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n0, ms0 = ctx.timing_read(0)
    n1, ms1 = ctx.timing_read(1)
    ctx.timing_enable(0)
    # algorithmic bytes of a launch over its entries: each entry's fields and the
    # links once (entries of a workgroup share the link loads), summed over launches
    V = int(np.prod(wl.dims))
    link_b = V * 36 * 16                                  # float64 links
    fwd_steps = steps * sum(i.k_used for i in infos)
    bwd_steps = steps * sum(max(i.k_used - 1, 0) for i in infos)
    f_b = ctx.kernel_bytes(0) - link_b
    b_b = ctx.kernel_bytes(1) - link_b
    fwd_bytes = f_b * fwd_steps + link_b * n0
    bwd_bytes = b_b * bwd_steps + link_b * n1
    picks = ctx.pair_ns()
    ctx.close()
    log(f"bench: fp64 batch {steps * n / dt:.2f} sources/s")
    which = 0 if ms0 >= ms1 else 1
    nl, ms, byt = (n0, ms0, fwd_bytes) if which == 0 else (n1, ms1, bwd_bytes)
    per_launch = byt / nl
    achieved = per_launch / (ms / nl * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(which), "kernel": KERNEL_NAMES[which],
                "bytes_per_launch": per_launch, "launches": nl, "mean_us": ms / nl * 1e3,
                "other_pair": {"kernel": KERNEL_NAMES[1 - which],
                               "achieved": ((bwd_bytes if which == 0 else fwd_bytes) / ((ms1 if which == 0 else ms0)
                                                                                         * 1e-3) / 1e9),
                               "mean_us": (ms1 / n1 if which == 0 else ms0 / n0) * 1e3,
                               "launches": n1 if which == 0 else n0,
                               "bytes_per_launch": (bwd_bytes / n1 if which == 0 else fwd_bytes / n0)}}

    # the reduced-precision batches on the same sources, each with its errors
    for prec, key in (("fp32links", "fp32_links_batched"), ("mixed", "fp32_vectors_batched")):
        ctx = Context(wl.dims, wl.mass, wl.mu, precision=prec)
        ctx.set_links(U)
        ctx.sign_grad_batched(eta, psi, ks, want_y=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sm, dUm, _, _, ym = ctx.sign_grad_batched(eta, psi, ks, want_y=True)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        ctx.close()
        out[key] = {"sources_per_s": n / dtm, "rel_err_vs_fp64": batch_errors(Sm, dUm, ym, S64, dU64, y64)}
        log(f"bench: {prec} batch {n / dtm:.2f} sources/s, errors vs fp64 {out[key]['rel_err_vs_fp64']}")
        del dUm, ym
    del dU64, y64
    res = {"dt": dt, "n": n, "ks": ks, "roofline": roofline, "infos": infos,
           "entries_per_workgroup": {"fwd_pair": picks[0], "bwd_pair": picks[1]}}
    res.update(out)
    return res


def single_8(steps: int = 20):
    """The 8^4 workload, one source per call, float64."""
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(2)
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    ctx = Context(wl.dims, wl.mass, wl.mu, precision="fp64")
    ctx.set_links(U)
    dU = torch.empty((4, wl.volume, 3, 3), dtype=torch.complex128, device="cuda")
    y = torch.empty((wl.volume, 4, 3), dtype=torch.complex128, device="cuda")
    for _ in range(3):
        ctx.sign_grad(eta, psi, wl.k, dU=dU, want_y=True)
    torch.cuda.synchronize()
    ctx.timing_enable(TIMING_EVERY)
    ctx.timing_read(0)
    ctx.timing_read(1)
    t0 = time.perf_counter()
    for _ in range(steps):
        S, _, _, info, _ = ctx.sign_grad(eta, psi, wl.k, dU=dU, want_y=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n0, ms0 = ctx.timing_read(0)
    n1, ms1 = ctx.timing_read(1)
    ctx.timing_enable(0)
    b1 = ctx.kernel_bytes(1)
    ctx.close()
    del y
    return {"workload": "8^4 (V=4096), mu=0.2, link spread 0.4, k=200, one Z2 source, fp64",
            "sources_per_s": steps / dt, "k_used": info.k_used, "newton_iters": info.newton_iters,
            "fwd_pair_mean_us": ms0 / max(n0, 1) * 1e3, "bwd_pair_mean_us": ms1 / max(n1, 1) * 1e3,
            "bwd_pair_GBs_cache_resident": b1 / (ms1 / max(n1, 1) * 1e-3) / 1e9}


def precision_14():
    """14^4 workload, k = 400: float64, float32 links and float32 vectors, one source."""
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(3)
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    out = {"workload": "14^4 (V=38416), mu=0.3, link spread 0.35, k=400, one Z2 source"}
    res = {}
    for prec in ("fp64", "fp32links", "mixed"):
        ctx = Context(wl.dims, wl.mass, wl.mu, precision=prec)
        ctx.set_links(U)
        ctx.sign_grad(eta, psi, wl.k, want_y=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S, dU, _, info, y = ctx.sign_grad(eta, psi, wl.k, want_y=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = (S, dU, y)
        out[f"{prec}_sources_per_s"] = 1.0 / dt
        if prec == "fp64":
            out["min_abs_re_ritz"] = info.min_abs_re_ritz
            out["biorth_err"] = info.biorth_err
            out["newton_iters"] = info.newton_iters
        ctx.close()
    # the nested projected-matrix step (inner size 100) against the plain one: the
    # sign alone, its dense-step time and the change of the result
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(U)
    nest = {}
    for m in (0, 100):
        ctx.set_nested(m)
        for _ in range(2):
            y, info = ctx.sign(psi, wl.k)
        torch.cuda.synchronize()
        nest[m] = (y, info.ms[1], info.ms[5])
    ctx.close()
    out["nested_m100"] = {"dense_ms_plain": nest[0][1], "dense_ms_nested": nest[100][1],
                          "sign_ms_plain": nest[0][2], "sign_ms_nested": nest[100][2],
                          "rel_diff_y": rel_t(nest[100][0], nest[0][0])}
    S64, dU64, y64 = res["fp64"]
    for prec in ("fp32links", "mixed"):
        S, dU, y = res[prec]
        out[f"{prec}_rel_err_vs_fp64"] = {"y": rel_t(y, y64), "S": abs(S - S64) / abs(S64), "dU": rel_t(dU, dU64)}
    return out


def stencil_large():
    import torch
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import KERNEL_APPLY
    dims = (32, 32, 32, 32)
    V = 32 ** 4
    g = torch.Generator(device="cuda").manual_seed(1604)
    U = torch.randn((4, V, 3, 3), dtype=torch.complex128, device="cuda", generator=g)
    x = torch.randn((V, 4, 3), dtype=torch.complex128, device="cuda", generator=g)
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(U)
    for _ in range(3):
        ctx.apply_h(x)
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    ctx.timing_read(KERNEL_APPLY)
    for _ in range(20):
        ctx.apply_h(x)
    n, ms = ctx.timing_read(KERNEL_APPLY)
    b = ctx.kernel_bytes(KERNEL_APPLY)
    ctx.close()
    gbs = b / (ms / n * 1e-3) / 1e9
    return {"lattice": "32^4", "kernel": "k_apply_tmarch<double, double>", "bytes_per_launch": b,
            "mean_ms": ms / n, "achieved_GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def host_description():
    cpu = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]
    except Exception:   # noqa: BLE001 - the description is best effort
        pass
    return cpu, blas


def cpu_baseline(k_sample: int, k_mean: float):
    """The oracle (torch-CPU float64 forward TSL + autograd all-links gradient) on
    source 0 of the 6x18^3 batch at a bounded Krylov size, scaled to a source of
    the batch's mean Krylov size (the oracle's cost grows linearly in k)."""
    import torch
    from oracle import grad as GR
    from oracle.wilson import WilsonOperator
    from synthetic import workload
    wl = workload(4)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi()[0], wl.eta()[0]
    t0 = time.perf_counter()
    GR.grad_autograd(op, U, psi, eta, k_sample)
    dt = time.perf_counter() - t0
    per_source = dt * k_mean / k_sample
    cpu, blas = host_description()
    return {"value": 1.0 / per_source, "unit": "sources/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"source 0 of the 6x18^3 batch at k={k_sample}: forward TSL + torch-CPU autograd dS/dU, "
                      f"{dt:.1f} s, scaled by {k_mean:.1f}/{k_sample} to the batch's mean Krylov size",
            "affinity_cpus": len(os.sched_getaffinity(0)), "torch_threads": torch.get_num_threads(),
            "blas": blas, "cpu_model": cpu}


def copy_probe():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"bench: copy probe of {n} bytes done (3 launches)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 8^4, 14^4 and 32^4 legs")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the single-GPU path is what this "
              f"library implements", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
    log(f"bench: 6x18^3 batch of 32 sources, warmup {args.warmup}, steps {args.steps}")
    h = headline(args.steps, args.warmup)
    n, dt = h["n"], h["dt"]
    out = {"metric": METRIC, "value": args.steps * n / dt, "unit": "sources/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "6x18^3 batching workload (V=34992, n=419904), Wilson mass -2, mu=0.5, "
                                  "SU(3) link spread 0.35, 32 Z2 sources, k uniform in [100, 400]; per source "
                                  "sgn(H)psi and all-links dS/dU of Re<eta|sgn(H)|psi>, one batched call per step",
                      "lattice": "18x18x18x6", "sources": n, "sum_k": int(sum(h["ks"])),
                      "precision": "float64 links, Krylov vectors, stencil arithmetic, accumulation, inner "
                                   "products and dense sign/Frechet step (bit-identical to the single-source path)",
                      "k_used": [i.k_used for i in h["infos"]],
                      "entries_per_workgroup": h["entries_per_workgroup"]},
           "fp64_single_source_sources_per_s": h["fp64_single_source_sources_per_s"],
           "fp64_batch_identical_to_single_k_ge_300": h["fp64_batch_identical_to_single_k_ge_300"],
           "speedup_vs_fp64_single_source": (args.steps * n / dt) / h["fp64_single_source_sources_per_s"],
           "fp32_links_batched": h["fp32_links_batched"],
           "fp32_vectors_batched": h["fp32_vectors_batched"],
           "roofline": h["roofline"]}
    if not args.no_extras:
        out["single_8x8x8x8"] = single_8()
        log(f"bench: 8^4 single source {out['single_8x8x8x8']['sources_per_s']:.2f} sources/s")
        out["precision_14x14x14x14"] = precision_14()
        log(f"bench: 14^4 fp64 {out['precision_14x14x14x14']['fp64_sources_per_s']:.2f} sources/s")
        out["stencil_large"] = stencil_large()
        log(f"bench: 32^4 stencil {out['stencil_large']['achieved_GBs']:.0f} GB/s")
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample (~10-20 s)")
        out["cpu_baseline"] = cpu_baseline(120, sum(h["ks"]) / n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
