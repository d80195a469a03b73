"""GPU batched derivative (many sources, uneven Krylov sizes) and the link-current estimator.

* every source of a batch gives bit-for-bit the single-source result (the
  kernels reduce in a fixed order per source, whatever else shares the launch),
  at the 4^4 workload (k = 64, 17, 40, 64, 1), at 8^4 (k from 150 to 200) and
  on a 10^4 lattice, which runs the colour-split stencil layout on an
  XCD-ordered, padded grid (k = 40, 25, 33, with the oracle for one source);
* on that layout, 1, 2 or 4 entries per workgroup and the timed pick give the
  same bits (five entries: a ragged last workgroup);
* against the oracle per source: S, dS/dU, dS/dpsi to 1e-10 relative;
* a zero source inside a batch: S = 0 and zero derivatives, the others unchanged; on
  the colour-split lattice with one, two and four entries per workgroup, all giving the
  same bits;
* the current estimator against the oracle estimator (mean of per-source U(1)
  projections of autograd gradients, eta = g5 xi): j to 1e-10 relative,
  divergence and total current to 1e-10 of max |j|, the per-sample Ward
  residual below 1e-10;
* more sources than one launch serves (70 > 64): the estimator accumulates over
  consecutive groups and still matches the oracle;
* the deflated estimator (10 eigenpairs of the dense H, the eigenpairs' motion in
  every term) against the oracle's, and its Ward residual over 70 sources.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import current as CU
from oracle import grad as GR
from oracle.wilson import WilsonOperator
from synthetic import random_links, workload, z2_complex_source

pytestmark = pytest.mark.gpu


def _ctx(dims, mass, mu, U):
    from paper_1604_08057_amd import Context
    ctx = Context(dims, mass, mu)
    ctx.set_links(dev(U))
    return ctx


def _sources(n, V, seed):
    r = np.random.default_rng(seed)
    return np.stack([z2_complex_source(V, r) for _ in range(n)])


def _batch_vs_single(dims, mass, mu, U, psis, etas, ks):
    ctx = _ctx(dims, mass, mu, U)
    S, dU, dpsi, infos = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_dpsi=True)
    for s, k in enumerate(ks):
        S1, dU1, dpsi1, info1 = ctx.sign_grad(dev(etas[s]), dev(psis[s]), k, want_dpsi=True)
        assert infos[s].k_used == info1.k_used
        assert S[s] == S1, (s, S[s], S1)
        assert torch.equal(dU[s], dU1), s
        assert torch.equal(dpsi[s], dpsi1), s
    ctx.close()
    return S, host(dU), host(dpsi), infos


def test_batch_equals_single_and_oracle_4():
    wl = workload(1)
    U = wl.links()
    ks = [64, 17, 40, 64, 1]
    psis, etas = _sources(5, 256, 41), _sources(5, 256, 42)
    say(f"batched 4^4 ks={ks}")
    S, dU, dpsi, infos = _batch_vs_single(wl.dims, wl.mass, wl.mu, U, psis, etas, ks)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    for s, k in enumerate(ks):
        ref = GR.grad_autograd(op, U, psis[s], etas[s], k)
        eS = abs(S[s] - ref["S"]) / abs(ref["S"])
        # k = 1: sgn(alpha_1) psi does not depend on the links (G = 0 exactly)
        eG = rel(dU[s], ref["G"]) if np.any(ref["G"]) else np.abs(dU[s]).max() / abs(ref["S"])
        eP = rel(dpsi[s], ref["dpsi"])
        say(f"  source {s} k={k}: S {eS:.2e} G {eG:.2e} dpsi {eP:.2e}")
        assert infos[s].k_used == ref["k_used"]
        assert eS < 1e-10 and eG < 1e-10 and eP < 1e-10


def test_batch_equals_single_8():
    wl = workload(2)
    ks = [200, 150, 187, 163]
    say(f"batched 8^4 ks={ks}")
    _batch_vs_single(wl.dims, wl.mass, wl.mu, wl.links(), _sources(4, 4096, 43), _sources(4, 4096, 44), ks)


def test_batch_equals_single_colour_split():
    dims, mass, mu = (10, 10, 10, 10), -2.0, 0.3
    U = random_links(dims, 0.4, np.random.default_rng(9))
    ks = [40, 25, 33]
    psis, etas = _sources(3, 10000, 47), _sources(3, 10000, 48)
    say(f"batched 10^4 ks={ks}")
    S, dU, dpsi, infos = _batch_vs_single(dims, mass, mu, U, psis, etas, ks)
    ref = GR.grad_autograd(WilsonOperator(dims, mass, mu), U, psis[1], etas[1], ks[1])
    eS = abs(S[1] - ref["S"]) / abs(ref["S"])
    eG, eP = rel(dU[1], ref["G"]), rel(dpsi[1], ref["dpsi"])
    say(f"  source 1 vs oracle: S {eS:.2e} G {eG:.2e} dpsi {eP:.2e}")
    assert eS < 1e-10 and eG < 1e-10 and eP < 1e-10


def test_batch_pair_ns_identical():
    # the colour-split pair kernels with 1, 2 or 4 entries per workgroup (sharing
    # every link load) and the timed pick give the same bits; five entries leave a
    # ragged last workgroup for 2 and 4, and the list shrinks as entries finish
    dims, mass, mu = (10, 10, 10, 10), -2.0, 0.3
    U = random_links(dims, 0.4, np.random.default_rng(19))
    ks = [30, 12, 27, 30, 19]
    psis, etas = _sources(5, 10000, 49), _sources(5, 10000, 50)
    ctx = _ctx(dims, mass, mu, U)
    runs = {}
    for ns in (0, 1, 2, 4):
        say(f"batched 10^4 ks={ks} entries per workgroup {ns or 'timed'}")
        ctx.set_pair_ns(ns)
        S, dU, dpsi, _ = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_dpsi=True)
        runs[ns] = (S, dU, dpsi)
    fwd, bwd = ctx.pair_ns()
    say(f"  timed picks: forward {fwd}, reverse {bwd}")
    ctx.close()
    assert fwd in (1, 2, 4) and bwd in (1, 2, 4)
    S0, dU0, dpsi0 = runs[1]
    for ns in (0, 2, 4):
        S, dU, dpsi = runs[ns]
        assert S == S0, ns
        assert torch.equal(dU, dU0) and torch.equal(dpsi, dpsi0), ns


def test_pair_ns_rejects_bad_value():
    from paper_1604_08057_amd.tslov import TslovError
    ctx = _ctx((2, 2, 2, 4), -2.0, 0.3, random_links((2, 2, 2, 4), 0.5, np.random.default_rng(1)))
    with pytest.raises(TslovError):
        ctx.set_pair_ns(3)
    ctx.close()


def test_zero_source_in_batch():
    dims = (2, 2, 2, 4)
    r = np.random.default_rng(5)
    U = random_links(dims, 0.5, r)
    psis, etas = _sources(3, 32, 6), _sources(3, 32, 7)
    psis[1] = 0.0
    ctx = _ctx(dims, -2.0, 0.3, U)
    S, dU, dpsi, infos = ctx.sign_grad_batched(dev(etas), dev(psis), [12, 9, 7], want_dpsi=True)
    assert S[1] == 0.0 and infos[1].k_used == 0
    assert torch.count_nonzero(dU[1]).item() == 0 and torch.count_nonzero(dpsi[1]).item() == 0
    for s, k in ((0, 12), (2, 7)):
        S1, dU1, _, _ = ctx.sign_grad(dev(etas[s]), dev(psis[s]), k)
        assert S[s] == S1 and torch.equal(dU[s], dU1)
    ctx.close()


def _current_case(dims, mass, mu, U, xis, ks, tag):
    op = WilsonOperator(dims, mass, mu)
    jr, _ = CU.current_tsl(op, U, xis, ks)
    dr, tr = CU.divergence(jr, op)
    ctx = _ctx(dims, mass, mu, U)
    j, div, tot, ward, infos = ctx.current_estimate(dev(xis), ks)
    ctx.close()
    j, div, tot = host(j), host(div), host(tot)
    scale = np.abs(jr).max()
    ej = rel(j, jr)
    ed, et = np.abs(div - dr).max() / scale, np.abs(tot - tr).max() / scale
    say(f"  {tag}: j {ej:.2e} div {ed:.2e} tot {et:.2e} ward {ward:.2e} "
        f"(max|div| {np.abs(dr).max() / scale:.2e}, max|tot| {np.abs(tr).max() / scale:.2e} of max|j|)")
    assert ej < 1e-10 and ed < 1e-10 and et < 1e-10
    assert ward < 1e-10


def test_current_estimate_4():
    wl = workload(1)
    ks = [64, 30, 47, 12]
    say(f"current estimator 4^4 ks={ks}")
    _current_case(wl.dims, wl.mass, wl.mu, wl.links(), _sources(4, 256, 45), ks, "4^4")


def test_current_estimate_many_groups():
    dims = (2, 2, 2, 4)
    r = np.random.default_rng(8)
    U = random_links(dims, 0.5, r)
    n = 70
    ks = list(r.integers(4, 13, size=n))
    say(f"current estimator 2x2x2x4, {n} sources")
    _current_case(dims, -2.0, 0.3, U, _sources(n, 32, 46), ks, "70 sources")


@pytest.mark.parametrize("nsrc", [3, 70])
def test_current_estimate_deflated(nsrc):
    """The deflated estimator (l = 10 on 2^3x4) against oracle.current.current_deflated:
    j, divergence and total current to 1e-10, the deflated samples' Ward residual below
    1e-9; 70 sources run the Ward check in two chunks."""
    from oracle import deflation as DF
    from oracle.wilson import dense_h
    dims, mass, mu, l = (2, 2, 2, 4), -2.0, 0.3, 10
    r = np.random.default_rng(49)
    U = random_links(dims, 0.5, r)
    xis = _sources(nsrc, 32, 50)
    ks = [int(v) for v in r.integers(8, 25, size=nsrc)]
    lam, R, L = DF.eigenpairs(dense_h(U, dims, mass, mu), l)
    op = WilsonOperator(dims, mass, mu)
    sub = min(nsrc, 6)   # the oracle's deflated gradients take about a second per source
    jr = CU.current_deflated(U, xis[:sub], ks[:sub], dims, mass, mu, l)
    dr, tr = CU.divergence(jr, op)
    ctx = _ctx(dims, mass, mu, U)
    defl = ctx.deflation(dev(R.T.reshape(l, 32, 4, 3)), dev(L.T.reshape(l, 32, 4, 3)), lam)
    j, div, tot, ward, infos = ctx.current_estimate(dev(xis[:sub]), ks[:sub], defl=defl)
    scale = np.abs(jr).max()
    ej = rel(host(j), jr)
    ed, et = np.abs(host(div) - dr).max() / scale, np.abs(host(tot) - tr).max() / scale
    say(f"  deflated current ({sub} sources): j {ej:.2e} div {ed:.2e} tot {et:.2e} ward {ward:.2e} "
        f"cg iterations {infos[0].cg_iters}")
    assert ej < 1e-10 and ed < 1e-10 and et < 1e-10 and ward < 1e-9
    if nsrc > sub:
        j2, _, _, ward2, _ = ctx.current_estimate(dev(xis), ks, defl=defl)
        say(f"  deflated current ({nsrc} sources): Ward residual {ward2:.2e}")
        assert ward2 < 1e-9
    ctx.close()


def test_zero_source_colour_split_every_shape():
    """A zero source inside a batch on the colour-split lattice (10^4): it stops at the
    first step, and with two or four entries per workgroup its workgroups keep running
    for the others (its slots masked out of the LDS exchange).  Every shape gives the
    bits of one entry per workgroup, the zero source S = 0 and zero derivatives, and
    each other source the bits of its single-source call."""
    dims, mass, mu = (10, 10, 10, 10), -2.0, 0.3
    U = random_links(dims, 0.4, np.random.default_rng(29))
    ks = [20, 14, 18, 20, 9]
    psis, etas = _sources(5, 10000, 51), _sources(5, 10000, 52)
    psis[2] = 0.0
    ctx = _ctx(dims, mass, mu, U)
    runs = {}
    for ns in (1, 2, 4):
        ctx.set_pair_ns(ns)
        S, dU, dpsi, infos = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_dpsi=True)
        say(f"batched 10^4 with a zero source, entries per workgroup {ns}: k_used {[i.k_used for i in infos]}")
        assert S[2] == 0.0 and infos[2].k_used == 0
        assert torch.count_nonzero(dU[2]).item() == 0 and torch.count_nonzero(dpsi[2]).item() == 0
        runs[ns] = (S, dU, dpsi)
    ctx.set_pair_ns(1)
    for s in (0, 3, 4):
        S1, dU1, _, _ = ctx.sign_grad(dev(etas[s]), dev(psis[s]), ks[s])
        assert runs[1][0][s] == S1 and torch.equal(runs[1][1][s], dU1), s
    ctx.close()
    S0, dU0, dpsi0 = runs[1]
    for ns in (2, 4):
        S, dU, dpsi = runs[ns]
        assert S == S0, ns
        assert torch.equal(dU, dU0) and torch.equal(dpsi, dpsi0), ns
