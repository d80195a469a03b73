"""GPU parity at the full lattice sizes of the precision and batching workloads.

Launches here span more workgroups than the chip has compute units (up to 547
stencil workgroups per source at 6x18^3), the regime in which the small-lattice
tests cannot show a defect of the field accessors.  Checked on sampled sources
that the oracle computes one by one:

* 6x18^3 (V = 34992, mu = 0.5): sgn(H)psi at k = 40 and k = 149 (source 0's
  Krylov size in the batch) against the oracle TSL to 1e-10 relative, and
  bit-identical on a repeated call;
* 6x18^3 batched derivative: the two sampled sources of the 32-source batch
  with the smallest Krylov sizes
  (run in one batched call) against torch autograd through the oracle TSL, S,
  dS/dU to max(1e-10, 10 sigma), sigma the oracle's own change under a
  permuted summation order; the U(1) Ward identity per site on the GPU outputs;
* 14x14^3 (V = 38416): sgn(H)psi at k = 100 against the oracle;
* 14x14^3 at its Krylov size k = 400 (float64): y at 64 sampled sites, |y|, S,
  D_ov psi, the smallest |Re theta| and the biorthogonality probe against the
  oracle's values stored by tests/golden/make_large_refs.py (its TSL takes a
  minute per run), to max(1e-10, 10 sigma); dS/dU by Richardson-extrapolated
  central differences of the GPU forward along 32 link directions; the U(1) Ward
  identity at every site; Krylov-vector recompute in segments of 20 against the
  stored-vector run; the float32-link variant against the stored oracle run on
  the rounded links (parity) and against float64 (stated error); the float32
  variant's stated error and flag;
* the whole 32-source 6x18^3 batch (k from 100 to 400) in one call: the largest-k
  source's S and y against the stored oracle; the per-sample Ward identity of
  all 32 sources (the current estimator's residual) below 1e-9; a k >= 300 source
  of the batch bit-identical to its single-source call.
"""
import os

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle.wilson import WilsonOperator
from synthetic import config_rng, workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with np.load(os.path.join(GOLDEN, name + ".npz")) as z:
        return {k: z[k] for k in z.files}


def _sampled(y, sites):
    return y.reshape(-1, 12)[sites].reshape(len(sites), 4, 3)


def _ctx(wl):
    from paper_1604_08057_amd import Context
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(wl.links()))
    return ctx


@pytest.mark.parametrize("k", [40, 149])
def test_sign_batching_lattice(k):
    wl = workload(4)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    psi = wl.psi()[0]
    say(f"sign 6x18^3 k={k}")
    ref = GR.forward(op, wl.links(), psi, k)
    ctx = _ctx(wl)
    y1, info = ctx.sign(dev(psi), k)
    y2, _ = ctx.sign(dev(psi), k)
    ctx.close()
    e = rel(host(y1), ref["y"])
    say(f"  k_used={info.k_used} y err {e:.2e}")
    assert torch.equal(y1, y2)
    assert info.k_used == ref["k_used"] and e < 1e-10


def test_batched_grad_batching_lattice_sampled():
    wl = workload(4)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U = wl.links()
    psis, etas = wl.psi(), wl.eta()
    ks = [int(k) for k in wl.krylov_sizes()]
    # the two smallest Krylov sizes: the oracle's autograd tape grows with k
    # (about 0.7 GB of host memory per step at this volume)
    pick = [int(i) for i in np.argsort(ks, kind="stable")[:2]]
    say(f"batched grad 6x18^3, sampled sources {pick} with k={[ks[s] for s in pick]}")
    ctx = _ctx(wl)
    S, dU, dpsi, infos = ctx.sign_grad_batched(dev(etas[pick]), dev(psis[pick]), [ks[s] for s in pick],
                                               want_dpsi=True)
    y = [host(ctx.sign(dev(psis[s]), ks[s])[0]) for s in pick]
    ctx.close()
    perm = np.random.default_rng(0).permutation(12 * op.volume)
    for i, s in enumerate(pick):
        ref = GR.grad_autograd(op, U, psis[s], etas[s], ks[s])
        alt = GR.grad_autograd(op, U, psis[s], etas[s], ks[s], perm=perm)
        sig_S = abs(alt["S"] - ref["S"]) / abs(ref["S"])
        sig_G = rel(alt["G"], ref["G"])
        eS = abs(S[i] - ref["S"]) / abs(ref["S"])
        eG = rel(host(dU[i]), ref["G"])
        say(f"  source {s}: S err {eS:.2e} (sigma {sig_S:.2e}) G err {eG:.2e} (sigma {sig_G:.2e})")
        assert infos[i].k_used == ref["k_used"]
        assert eS < max(1e-10, 10 * sig_S) and eG < max(1e-10, 10 * sig_G)
        lhs, rhs = GR.ward_residual(op, host(dU[i]), U, psis[s], etas[s], y[i], host(dpsi[i]))
        say(f"  ward max |lhs - rhs| / max |lhs| = {np.abs(lhs - rhs).max() / np.abs(lhs).max():.2e}")
        assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(lhs).max()


def test_sign_precision_lattice():
    wl = workload(3)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    psi = wl.psi()
    k = 100
    say(f"sign {wl.dims} k={k}")
    ref = GR.forward(op, wl.links(), psi, k)
    ctx = _ctx(wl)
    y, info = ctx.sign(dev(psi), k)
    ctx.close()
    e = rel(host(y), ref["y"])
    say(f"  y err {e:.2e}")
    assert e < 1e-10


def test_precision_lattice_full_krylov_size():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import FLAG_GRAD_FP32_VECTORS
    wl = workload(3)
    g = _golden("precision_14x14x14x14_k400")
    sites = g["sites"]
    psi, eta = wl.psi(), wl.eta()
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    res = {}
    for prec in ("fp64", "fp32links", "mixed"):
        ctx = Context(wl.dims, wl.mass, wl.mu, precision=prec)
        ctx.set_links(dev(wl.links()))
        y, info = ctx.sign(dev(psi), wl.k)
        d, _ = ctx.overlap(dev(psi), wl.k)
        S, dU, dpsi, ginfo = ctx.sign_grad(dev(eta), dev(psi), wl.k, want_dpsi=True)
        res[prec] = dict(y=host(y), d=host(d), info=info, S=S, G=host(dU), ginfo=ginfo)
        ctx.close()
        say(f"14^4 k=400 {prec}: k_used {info.k_used} S {S:.15e} min|Re theta| {info.min_abs_re_ritz:.4e} "
            f"biorth {info.biorth_err:.2e} ms {ginfo.ms[5]:.1f}")

    def check(prec, tag, tol):
        r = res[prec]
        ey = rel(_sampled(r["y"], sites), g["y_sites_" + tag])
        en = abs(np.linalg.norm(r["y"]) - g["norm_y_" + tag]) / g["norm_y_" + tag]
        eS = abs(r["S"] - g["S_" + tag]) / abs(g["S_" + tag])
        ed = rel(_sampled(r["d"], sites), _sampled(psi, sites) + g5 * g["y_sites_" + tag])
        say(f"  {prec} vs oracle ({tag} links): y(sites) {ey:.2e} |y| {en:.2e} S {eS:.2e} D_ov {ed:.2e}")
        return ey, en, eS, ed

    sig = max(float(g["sigma_y_fp64"]), float(g["sigma_S_fp64"]))
    tol = max(1e-10, 10 * sig)
    for prec, tag in (("fp64", "fp64"), ("fp32links", "fp32links")):
        assert res[prec]["info"].k_used == int(g["k_used_" + tag]) == wl.k
        errs = check(prec, tag, tol)
        assert max(errs) < tol, errs
        i = res[prec]["info"]
        assert abs(i.min_abs_re_ritz - float(g["min_abs_re_ritz_" + tag])) < 1e-9 * float(g["max_abs_ritz_" + tag])
        assert i.biorth_err < 1e-6 and float(g["biorth_" + tag]) < 1e-6
    # float32 links against the float64 truth: the stated per-output error
    e32 = check("fp32links", "fp64", 0)
    eG32 = rel(res["fp32links"]["G"], res["fp64"]["G"])
    say(f"  fp32links vs fp64: y {e32[0]:.2e} S {e32[2]:.2e} dU {eG32:.2e}")
    assert e32[0] < 1e-6 and e32[2] < 1e-6 and eG32 < 1e-4
    emx = check("mixed", "fp64", 0)
    eGm = rel(res["mixed"]["G"], res["fp64"]["G"])
    say(f"  mixed vs fp64: y {emx[0]:.2e} S {emx[2]:.2e} dU {eGm:.2e} flags {res['mixed']['ginfo'].flags}")
    assert emx[0] < 1e-3 and emx[2] < 1e-3
    assert res["mixed"]["ginfo"].flags & FLAG_GRAD_FP32_VECTORS


def test_precision_lattice_derivative():
    from paper_1604_08057_amd import Context
    wl = workload(3)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi(), wl.eta()
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(U))
    pe, pp = dev(eta), dev(psi)
    say("14^4 k=400 derivative: stored vs recompute(20), Ward, FD on 32 directions")
    S0, dU0, dp0, i0, y0 = ctx.sign_grad(pe, pp, wl.k, want_dpsi=True, want_y=True)
    S1, dU1, dp1, i1 = ctx.sign_grad(pe, pp, wl.k, want_dpsi=True, recompute=20)
    e, ep = rel(host(dU1), host(dU0)), rel(host(dp1), host(dp0))
    say(f"  recompute m=20: S equal {S1 == S0} dU {e:.2e} dpsi {ep:.2e} (ms {i0.ms[5]:.1f} / {i1.ms[5]:.1f})")
    assert S1 == S0 and e < 1e-12 and ep < 1e-12
    G = host(dU0)
    lhs, rhs = GR.ward_residual(op, G, U, psi, eta, host(y0), host(dp0))
    w = np.abs(lhs - rhs).max() / np.abs(lhs).max()
    say(f"  Ward identity: max |lhs - rhs| / max |lhs| = {w:.2e}")
    assert w < 1e-9

    def S_of(Uc):
        ctx.set_links(dev(Uc))
        y, _ = ctx.sign(pp, wl.k)
        return float(np.real(np.vdot(eta, host(y))))

    r = config_rng(3, 4)
    ad, fd = [], []
    for i in range(16):
        nu, site = int(r.integers(0, 4)), int(r.integers(0, wl.volume))
        for X in (GR.su3_direction(r), np.eye(3, dtype=complex)):
            ad.append(GR.directional_from_gradient(G, U, nu, site, X))
            f1 = GR.fd_directional(S_of, U, nu, site, X, 2e-3)
            f2 = GR.fd_directional(S_of, U, nu, site, X, 1e-3)
            fd.append((4 * f2 - f1) / 3)
    ctx.close()
    ad, fd = np.array(ad), np.array(fd)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    say(f"  FD on 32 link directions: rel err {err:.2e} (|fd| {np.linalg.norm(fd):.3e})")
    assert err < 1e-6


def test_batching_whole_batch():
    from paper_1604_08057_amd import Context
    wl = workload(4)
    g = _golden("batching_6x18x18x18_kmax")
    psis, etas = wl.psi(), wl.eta()
    ks = [int(k) for k in wl.krylov_sizes()]
    s_max = int(g["source"])
    assert ks[s_max] == int(g["k"]) == max(ks)
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(wl.links()))
    say(f"whole 6x18^3 batch: 32 sources, k from {min(ks)} to {max(ks)}")
    S, dU, _, infos, y = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_y=True)
    ey = rel(_sampled(host(y[s_max]), g["sites"]), g["y_sites"])
    eS = abs(S[s_max] - float(g["S"])) / abs(float(g["S"]))
    tol = max(1e-10, 10 * max(float(g["sigma_y"]), float(g["sigma_S"])))
    say(f"  largest-k source {s_max} (k={ks[s_max]}): y(sites) {ey:.2e} S {eS:.2e} (tol {tol:.1e}) "
        f"min|Re theta| {infos[s_max].min_abs_re_ritz:.3e} biorth {infos[s_max].biorth_err:.2e}")
    assert infos[s_max].k_used == int(g["k_used"])
    assert ey < tol and eS < tol
    assert abs(infos[s_max].min_abs_re_ritz - float(g["min_abs_re_ritz"])) < 1e-9 * float(g["max_abs_ritz"])
    # a k >= 300 source alone gives the bits it gets inside the batch
    s1 = next(i for i in range(len(ks)) if ks[i] >= 300 and i != s_max)
    S1, dU1, _, _ = ctx.sign_grad(dev(etas[s1]), dev(psis[s1]), ks[s1])
    say(f"  source {s1} (k={ks[s1]}) alone vs in the batch: S equal {S1 == S[s1]}, "
        f"dU equal {bool(torch.equal(dU1, dU[s1]))}")
    assert S1 == S[s1] and torch.equal(dU1, dU[s1])
    del dU, y
    # the per-sample Ward identity of every source (eta = g5 xi, as the current estimator uses)
    j, div, tot, ward, cinfos = ctx.current_estimate(dev(psis), ks)
    ctx.close()
    say(f"  current estimator over 32 sources: Ward residual {ward:.2e}")
    assert ward < 1e-9
    assert all(ci.k_used == k for ci, k in zip(cinfos, ks))
