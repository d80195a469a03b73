"""GPU derivative of the deflated sign function (eigenpair motion) against the oracle.

The oracle differentiates the TSL part by autograd and the eigenpair part with
reduced resolvents built from the full dense spectrum; the GPU solves the
reduced-resolvent systems by CGNR to relative residual 1e-13.  Bar: S, dS/dU and
dS/dpsi to 1e-10 relative (the float64 bar).
Cases: l = 10 (k = 24) on 2^3x4 and l = 20 (k = 60) on 3^3x4, the latter also
with the Krylov vectors regenerated in segments of 11 steps; each with both
operator forms of the shifted solves (multi-right-hand-side, colour split,
matrix-core; the t-march form needs (x, y, z) volumes in multiples of 1024 sites and
runs the multi-right-hand-side form here).  Three sources in one batched deflated
call against the oracle and against their single-source calls.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import deflation as DF
from oracle.wilson import dense_h
from synthetic import random_links, z2_complex_source

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("dims,l,k,m", [((2, 2, 2, 4), 10, 24, 0), ((3, 3, 3, 4), 20, 60, 0),
                                        ((3, 3, 3, 4), 20, 60, 11)])
def test_deflated_gradient(dims, l, k, m, form):
    from paper_1604_08057_amd import Context
    mass, mu = -2.0, 0.3
    r = np.random.default_rng(31)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, r)
    psi, eta = z2_complex_source(V, r), z2_complex_source(V, r)
    H = dense_h(U, dims, mass, mu)
    lam, R, L = DF.eigenpairs(H, l)
    G, S, pb = DF.deflated_gradient(U, psi, eta, k, dims, mass, mu, l)
    ctx = Context(dims, mass, mu)
    ctx.set_links(dev(U))
    ctx.set_cg_operator(form)
    defl = ctx.deflation(dev(R.T.reshape(l, V, 4, 3)), dev(L.T.reshape(l, V, 4, 3)), lam)
    Sg, dU, dpsi, info = ctx.sign_grad(dev(eta), dev(psi), k, want_dpsi=True, defl=defl, recompute=m)
    ctx.close()
    eS, eG, eP = abs(Sg - S) / abs(S), rel(host(dU), G), rel(host(dpsi), pb)
    say(f"deflated grad {dims} l={l} k={k} recompute={m} form={form}: S {eS:.2e} G {eG:.2e} dpsi {eP:.2e} cg iterations {info.cg_iters}")
    assert eS < 1e-10 and eG < 1e-10 and eP < 1e-10


def test_batched_deflated_gradient():
    """Three sources with uneven Krylov sizes in one batched deflated call (l = 10 on
    2^3x4): each source against the oracle (S, dS/dU, dS/dpsi to 1e-10) and equal bit for
    bit to its single-source call (the batched shifted solves keep each system's
    arithmetic)."""
    from paper_1604_08057_amd import Context
    dims, l, ks = (2, 2, 2, 4), 10, [24, 18, 30]
    mass, mu = -2.0, 0.3
    r = np.random.default_rng(33)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, r)
    psis = np.stack([z2_complex_source(V, r) for _ in ks])
    etas = np.stack([z2_complex_source(V, r) for _ in ks])
    lam, R, L = DF.eigenpairs(dense_h(U, dims, mass, mu), l)
    ctx = Context(dims, mass, mu)
    ctx.set_links(dev(U))
    defl = ctx.deflation(dev(R.T.reshape(l, V, 4, 3)), dev(L.T.reshape(l, V, 4, 3)), lam)
    S, dU, dpsi, infos, y = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_dpsi=True, want_y=True, defl=defl)
    for s, k in enumerate(ks):
        G, Sr, pb = DF.deflated_gradient(U, psis[s], etas[s], k, dims, mass, mu, l)
        eS, eG, eP = abs(S[s] - Sr) / abs(Sr), rel(host(dU[s]), G), rel(host(dpsi[s]), pb)
        S1, dU1, dp1, i1, y1 = ctx.sign_grad(dev(etas[s]), dev(psis[s]), k, want_dpsi=True, want_y=True, defl=defl)
        same = S1 == S[s] and torch.equal(dU1, dU[s]) and torch.equal(dp1, dpsi[s]) and torch.equal(y1, y[s])
        say(f"batched deflated grad source {s} (k={k}): S {eS:.2e} G {eG:.2e} dpsi {eP:.2e}, "
            f"cg iterations {infos[s].cg_iters} (single {i1.cg_iters}), equal to single: {same}")
        assert eS < 1e-10 and eG < 1e-10 and eP < 1e-10
        assert same
    ctx.close()
