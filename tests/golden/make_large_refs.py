"""Write the oracle references of the full-size parity tests (tests/golden/*.npz).

Calls only ``oracle/`` and ``synthetic/``; run on the CPU:

    python tests/golden/make_large_refs.py

The oracle's TSL at these lattices takes one to two minutes per run, too long to
repeat inside every GPU test session, so the tests read what this script stored:
for each case the scalar S = Re eta^H y, |y|, the Ritz-value extremes of T_k,
the loss-of-biorthogonality probe |w_1^H v_k| + |w_k^H v_1|, and y at 64 sampled
sites (stream 4 of the case's seed scheme), together with the oracle's own
sensitivity to the summation order of its inner products (a second run with a
permuted order), which sets the parity tolerance.

Cases:
* ``precision_14x14x14x14_k400``: the 14^4 workload (mu = 0.3, spread 0.35), k = 400,
  on the float64 links and on the links rounded to float32 (what the float32-link
  variant of the library reads);
* ``batching_6x18x18x18_kmax``: the 6x18^3 workload (mu = 0.5), the source with the
  largest Krylov size of the 32-source batch.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import grad as GR  # noqa: E402
from oracle.wilson import WilsonOperator  # noqa: E402
from synthetic import config_rng, workload  # noqa: E402

NSAMPLE = 64


def _summary(op, U, psi, eta, k, sites, perm):
    t0 = time.time()
    f = GR.forward(op, U, psi, k)
    t1 = time.time()
    g = GR.forward(op, U, psi, k, perm=perm)
    y = f["y"]
    th = np.linalg.eigvals(f["T"])
    kk = f["k_used"]
    bi = f["biorth"]
    out = dict(S=np.real(np.vdot(eta, y)), norm_y=np.linalg.norm(y), y_sites=y[sites], k_used=kk,
               min_abs_re_ritz=np.abs(th.real).min(), max_abs_ritz=np.abs(th).max(), biorth=bi,
               sigma_y=np.linalg.norm(g["y"] - y) / np.linalg.norm(y),
               sigma_S=abs(np.real(np.vdot(eta, g["y"])) - np.real(np.vdot(eta, y))) / abs(np.real(np.vdot(eta, y))))
    print(f"  k_used {kk} S {out['S']:.15e} sigma_y {out['sigma_y']:.2e} min|Re theta| "
          f"{out['min_abs_re_ritz']:.3e} biorth {bi:.2e} ({t1 - t0:.0f} s per run)", flush=True)
    return out


def _save(name, d):
    np.savez(os.path.join(HERE, name + ".npz"), **{k: np.asarray(v) for k, v in d.items()})


def main():
    wl = workload(3)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi(), wl.eta()
    sites = np.sort(config_rng(3, 4).choice(wl.volume, NSAMPLE, replace=False))
    perm = np.random.default_rng(0).permutation(12 * wl.volume)
    print(f"14^4 k={wl.k} float64 links", flush=True)
    d64 = _summary(op, U, psi, eta, wl.k, sites, perm)
    print(f"14^4 k={wl.k} links rounded to float32", flush=True)
    U32 = U.astype(np.complex64).astype(np.complex128)
    d32 = _summary(op, U32, psi, eta, wl.k, sites, perm)
    out = {"sites": sites, "k": wl.k}
    out.update({k + "_fp64": v for k, v in d64.items()})
    out.update({k + "_fp32links": v for k, v in d32.items()})
    _save("precision_14x14x14x14_k400", out)

    wl = workload(4)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    ks = wl.krylov_sizes()
    s = int(np.argmax(ks))
    U, psi, eta = wl.links(), wl.psi()[s], wl.eta()[s]
    sites = np.sort(config_rng(4, 4).choice(wl.volume, NSAMPLE, replace=False))
    perm = np.random.default_rng(0).permutation(12 * wl.volume)
    print(f"6x18^3 source {s} k={ks[s]}", flush=True)
    d = _summary(op, U, psi, eta, int(ks[s]), sites, perm)
    out = {"sites": sites, "source": s, "k": int(ks[s])}
    out.update(d)
    _save("batching_6x18x18x18_kmax", out)


if __name__ == "__main__":
    main()
