#!/usr/bin/env python3
"""Benchmark of the TSL sign function + all-links derivative on one MI355X.

One step = one source: S = Re <eta|TSL_k(H(U), psi)>, sgn(H)psi by two-sided
Lanczos, and dS/dU over all 4V links (tslov_sign_grad), on the 8^4 workload
(V = 4096, n = 49152, Wilson mass -2, mu = 0.2, k = 200, FP64) with seeded
synthetic SU(3) links (spread 0.4) and Z2-complex sources resident in HBM.

The JSON line carries:
* value: sources/s of the FP64 path over the timed steps;
* roofline: the dominant stencil kernel's algorithmic bytes per launch over its
  mean duration, timed with HIP events on the library stream during the timed
  steps; traffic from the committed counter summary when it matches the kernel
  source;
* cpu_baseline: the CPU oracle (torch/NumPy float64; forward TSL + autograd
  gradient) on one source of the same workload, on the host cores;
* batched: the 6x18^3 batching workload (32 Z2 sources, k drawn from [100, 400],
  mu = 0.5), all sources in one tslov_sign_grad_batched call (FP64), beside the
  single-source FP64 path on the first four sources and the same batch with the
  float32-vector path (sources/s and its error against the FP64 batch);
* precision: the 14^4 workload (k = 400) single source, FP64, with the
  float32-vector path's error against it;
* mixed: the float32-vector path on the 8^4 workload (sources/s, errors vs FP64);
* graphs: the 8^4 step with its Lanczos loops launched and replayed as HIP
  graphs, both without kernel timing;
* stencil_large: the FP64 Wilson stencil alone on a 32^4 lattice (1.15 GB per
  application, above the 256 MB last-level cache) for the HBM-bound figure.
With --copy-probe a 1 GiB device-to-device copy runs first (HBM counter
calibration for rocprofv3 --pmc).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sgn(H)ψ+dU-derivative sources/s, mixed vs FP64 @≤1e-6 rel; stencil HBM GB/s"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "k_fwd_pair<double> (fused Lanczos stencil pair, colour grid, hops on two wavefronts, epilogue operands on a third)",
                1: "k_bwd_rb_cg<double> (reverse-mode stencil pair, colour grid, hops on two wavefronts, epilogue operands on a third)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stencil_pair_8x8x8x8.txt")
# live kernel timing samples every 16th launch of a class: an event pair adds ~5 us
# of dispatch latency, which on every launch would slow the timed step by ~25%
TIMING_EVERY = 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def read_traffic(which: int):
    """HBM bytes per launch of the given stencil pair kernel (0 forward, 1 reverse) from
    the committed counter summary, or None if absent or taken on a different kernel source."""
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
        return float(vals["hbm_bytes_per_launch" if which == 1 else "fwd_pair_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(ctx, eta, psi, k, steps, warmup, dU, timing=False):
    import torch
    for _ in range(warmup):
        ctx.sign_grad(eta, psi, k, dU=dU)
    torch.cuda.synchronize()
    if timing:
        ctx.timing_enable(TIMING_EVERY)
        ctx.timing_read(0)
        ctx.timing_read(1)
    t0 = time.perf_counter()
    for _ in range(steps):
        S, _, _, info = ctx.sign_grad(eta, psi, k, dU=dU)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if timing:
        ctx.timing_enable(0)
    return (t1 - t0), S, info


def graph_leg(steps: int = 20):
    """The 8^4 step with the Lanczos loops launched and replayed as HIP graphs (no
    kernel timing; the context on a side stream, which capture needs)."""
    import numpy as np
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(2)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    dU = torch.empty((4, wl.volume, 3, 3), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    out = {}
    for graphs in (False, True):
        with torch.cuda.stream(torch.cuda.Stream()):
            ctx = Context(wl.dims, wl.mass, wl.mu)
        torch.cuda.synchronize()
        ctx.set_links(U)
        ctx.set_graphs(graphs)
        dt, _, _ = time_steps(ctx, eta, psi, wl.k, steps, 2, dU)
        ctx.close()
        out["graph_sources_per_s" if graphs else "launched_sources_per_s"] = steps / dt
    return out


def cpu_baseline(wl):
    import torch
    from oracle import grad as GR
    from oracle.wilson import WilsonOperator
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi(), wl.eta()
    t0 = time.perf_counter()
    GR.grad_autograd(op, U, psi, eta, wl.k)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "sources/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"1 source of the same workload ({wl.dims[0]}^4, k={wl.k}): forward TSL + torch-CPU "
                      f"autograd dS/dU, {dt:.1f} s"}


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
    return {"lattice": "32^4", "kernel": "k_apply_tmarch<double>", "bytes_per_launch": b, "mean_ms": ms / n,
            "achieved_GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def rel_t(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def batched_leg(ks_single: int = 4):
    """32-source 6x18^3 workload in one batched FP64 call, and the single-source path."""
    import numpy as np
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    ks = [int(k) for k in wl.krylov_sizes()]
    ctx = Context(wl.dims, wl.mass, wl.mu, precision="fp64")
    ctx.set_links(U)
    # warm-up with the full batch: the workspace (about 16 GB per source at k = 400)
    # is allocated here, outside the timed call
    ctx.sign_grad_batched(eta, psi, ks)
    torch.cuda.synchronize()
    ctx.timing_enable(1)      # batched launches are long: timing every one costs < 1%
    ctx.timing_read(0)
    ctx.timing_read(1)
    t0 = time.perf_counter()
    S, dU, _, infos = ctx.sign_grad_batched(eta, psi, ks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n0, ms0 = ctx.timing_read(0)
    n1, ms1 = ctx.timing_read(1)
    ctx.timing_enable(0)
    # algorithmic bytes of a launch over n entries: the fields of every entry and the
    # links once (entries of a workgroup share the link loads), summed over launches
    steps = sum(i.k_used for i in infos)
    bsteps = sum(max(i.k_used - 1, 0) for i in infos)
    link_b = int(np.prod(wl.dims)) * 36 * 16
    b0, b1 = ctx.kernel_bytes(0) - link_b, ctx.kernel_bytes(1) - link_b
    fwd_gbs = (b0 * steps + link_b * n0) / (ms0 * 1e-3) / 1e9
    bwd_gbs = (b1 * bsteps + link_b * n1) / (ms1 * 1e-3) / 1e9
    picks = ctx.pair_ns()
    dU0 = dU[0].clone()
    t1 = time.perf_counter()
    for s in range(ks_single):
        Ss, dUs, _, _ = ctx.sign_grad(eta[s], psi[s], ks[s])
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    same = bool(torch.equal(dUs, dU0)) if ks_single == 1 else None
    ctx.close()
    # the same batch with the float32 stencil and vectors (FP64 dots, coefficients,
    # projected-matrix step and accumulation): throughput and error against FP64
    ctxm = Context(wl.dims, wl.mass, wl.mu, precision="mixed")
    ctxm.set_links(U)
    ctxm.sign_grad_batched(eta, psi, ks)
    torch.cuda.synchronize()
    tm = time.perf_counter()
    Sm, dUm, _, _ = ctxm.sign_grad_batched(eta, psi, ks)
    torch.cuda.synchronize()
    dtm = time.perf_counter() - tm
    ctxm.close()
    err_S = max(abs(a - b) / abs(b) for a, b in zip(Sm, S))
    errs = sorted(float(torch.linalg.vector_norm(dUm[s] - dU[s]) / torch.linalg.vector_norm(dU[s]))
                  for s in range(len(ks)))
    err_dU, med_dU = errs[-1], errs[len(errs) // 2]
    del dU, dUm
    return {"workload": "6x18^3 (V=34992), mu=0.5, link spread 0.35, 32 Z2 sources, k uniform in [100, 400]",
            "sources": len(ks), "sum_k": int(sum(ks)), "precision": "fp64",
            "sources_per_s": len(ks) / dt, "ms_per_call": dt * 1e3,
            "single_source_sources_per_s": ks_single / dt1, "single_source_sample": ks_single,
            "speedup_vs_single": (len(ks) / dt) / (ks_single / dt1),
            "fwd_pair_GBs": fwd_gbs, "fwd_pair_frac": fwd_gbs / HBM_PEAK_GBS,
            "bwd_pair_GBs": bwd_gbs, "bwd_pair_frac": bwd_gbs / HBM_PEAK_GBS,
            "launches": {"fwd_pair": n0, "bwd_pair": n1}, "identical_to_single": same,
            "entries_per_workgroup": {"fwd_pair": picks[0], "bwd_pair": picks[1]},
            "mixed_sources_per_s": len(ks) / dtm, "mixed_max_rel_err_S": err_S, "mixed_max_rel_err_dU": err_dU,
            "mixed_median_rel_err_dU": med_dU}


def precision_leg():
    """14^4 workload, k = 400: FP64 single source and the float32-vector path's error."""
    import numpy as np
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload
    wl = workload(3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    out = {"workload": "14^4 (V=38416), mu=0.3, link spread 0.35, k=400, one Z2 source"}
    res = {}
    for prec in ("fp64", "mixed"):
        ctx = Context(wl.dims, wl.mass, wl.mu, precision=prec)
        ctx.set_links(U)
        ctx.sign_grad(eta, psi, wl.k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S, dU, _, info = ctx.sign_grad(eta, psi, wl.k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        y, _ = ctx.sign(psi, wl.k)
        res[prec] = (S, dU, y)
        out[f"{prec}_sources_per_s"] = 1.0 / dt
        out[f"{prec}_newton_iters"] = info.newton_iters
        ctx.close()
    S64, dU64, y64 = res["fp64"]
    Sm, dUm, ym = res["mixed"]
    out["mixed_rel_err"] = {"y": rel_t(ym, y64), "S": abs(Sm - S64) / abs(S64), "dU": rel_t(dUm, dU64)}
    return out


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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched, precision, mixed and 32^4 legs")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the single-GPU path is what this "
              f"library implements", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1604_08057_amd import Context
    from synthetic import workload

    if args.copy_probe:
        copy_probe()
    wl = workload(2)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    ctx = Context(wl.dims, wl.mass, wl.mu, precision="fp64")
    ctx.set_links(U)
    dU = torch.empty((4, wl.volume, 3, 3), dtype=torch.complex128, device="cuda")
    log(f"bench: workload {wl.dims} k={wl.k} fp64, warmup {args.warmup}, steps {args.steps}")
    dt, S, info = time_steps(ctx, eta, psi, wl.k, args.steps, args.warmup, dU, timing=True)
    n0, ms0 = ctx.timing_read(0)
    n1, ms1 = ctx.timing_read(1)
    log(f"bench: {args.steps / dt:.2f} sources/s; fwd pair {n0} x {ms0 / max(n0, 1) * 1e3:.2f} us, "
        f"bwd pair {n1} x {ms1 / max(n1, 1) * 1e3:.2f} us")
    which = 0 if ms0 >= ms1 else 1
    n, ms = (n0, ms0) if which == 0 else (n1, ms1)
    per_launch = ctx.kernel_bytes(which)
    achieved = per_launch / (ms / n * 1e-3) / 1e9
    traffic = read_traffic(which)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": KERNEL_NAMES[which],
                "bytes_per_launch": per_launch, "launches": n, "mean_us": ms / n * 1e3}
    y64, _ = ctx.sign(psi, wl.k)
    dU64 = dU.clone()
    ctx.close()

    out = {"metric": METRIC, "value": args.steps / dt, "unit": "sources/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "sgn(H)psi + all-links dS/dU, 8^4 lattice (V=4096, n=49152), "
                                  "Wilson mass -2, mu=0.2, SU(3) link spread 0.4, k=200, one Z2 source",
                      "lattice": "8x8x8x8", "k": wl.k, "precision": "fp64", "k_used": info.k_used,
                      "newton_iters": info.newton_iters},
           "roofline": roofline}

    if not args.no_extras:
        ctxm = Context(wl.dims, wl.mass, wl.mu, precision="mixed")
        ctxm.set_links(U)
        dUm = torch.empty_like(dU)
        dtm, Sm, _ = time_steps(ctxm, eta, psi, wl.k, max(args.steps // 2, 1), 1, dUm)
        ym, _ = ctxm.sign(psi, wl.k)
        ctxm.close()
        out["mixed"] = {"sources_per_s": max(args.steps // 2, 1) / dtm, "precision": "float32 stencil and "
                        "vectors, float64 dots/coefficients/sign step/accumulation",
                        "rel_err_y_vs_fp64": rel_t(ym, y64), "rel_err_dU_vs_fp64": rel_t(dUm, dU64),
                        "rel_err_S_vs_fp64": abs(Sm - S) / abs(S)}
        log(f"bench: mixed {out['mixed']['sources_per_s']:.2f} sources/s")
        out["graphs"] = graph_leg()
        log(f"bench: 8^4 launched {out['graphs']['launched_sources_per_s']:.2f}, "
            f"graph-replayed {out['graphs']['graph_sources_per_s']:.2f} sources/s")
        out["batched"] = batched_leg()
        log(f"bench: batched 6x18^3 {out['batched']['sources_per_s']:.2f} sources/s "
            f"(single-source {out['batched']['single_source_sources_per_s']:.2f})")
        out["precision"] = precision_leg()
        log(f"bench: 14^4 fp64 {out['precision']['fp64_sources_per_s']:.2f} sources/s")
        out["stencil_large"] = stencil_large()
        log(f"bench: 32^4 stencil {out['stencil_large']['achieved_GBs']:.0f} GB/s")

    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on one source (~15-30 s)")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
