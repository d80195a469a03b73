"""Captured Lanczos loops (HIP graphs) against the launched loops.

The context runs on a side stream (capture needs a non-null stream).  Every
replay is checked bit for bit against the launched (eager) result, with eager
torch work and host synchronisations between the replays: the 8^4 colour-grid
layout (derivative calls: forward and reverse loops; the sign alone: forward
loop), a change of k (recapture) and back, and a batch on the 10^4
colour-split layout after its pair-kernel shape has been timed.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, say
from synthetic import random_links, workload, z2_complex_source

pytestmark = pytest.mark.gpu


def _side_stream_ctx(dims, mass, mu, U):
    from paper_1604_08057_amd import Context
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = Context(dims, mass, mu)
    torch.cuda.synchronize()
    ctx.set_links(U)
    return ctx


def _eager_noise(x):
    # unrelated work on the default stream between replays
    z = (x * 2.0).abs().sum()
    torch.cuda.synchronize()
    return z


def _same(a, b):
    return a[0] == b[0] and torch.equal(a[1], b[1]) and (a[2] is None or torch.equal(a[2], b[2]))


def test_graph_replays_match_eager_8():
    wl = workload(2)
    U, psi, eta = dev(wl.links()), dev(wl.psi()), dev(wl.eta())
    torch.cuda.synchronize()
    ctx = _side_stream_ctx(wl.dims, wl.mass, wl.mu, U)
    ref60 = ctx.sign_grad(eta, psi, 60, want_dpsi=True)
    ref45 = ctx.sign_grad(eta, psi, 45, want_dpsi=True)
    yref, _ = ctx.sign(psi, 60)
    ctx.set_graphs(True)
    for rep in range(3):
        say(f"graph 8^4 derivative k=60, call {rep} ({'capture' if rep == 0 else 'replay'})")
        assert _same(ctx.sign_grad(eta, psi, 60, want_dpsi=True), ref60), rep
        _eager_noise(psi)
    say("graph 8^4 derivative k=45 (recapture), then k=60 (recapture)")
    assert _same(ctx.sign_grad(eta, psi, 45, want_dpsi=True), ref45)
    assert _same(ctx.sign_grad(eta, psi, 60, want_dpsi=True), ref60)
    for rep in range(3):
        say(f"graph 8^4 sign k=60, call {rep}")
        y, _ = ctx.sign(psi, 60)
        assert torch.equal(y, yref), rep
        _eager_noise(y)
    ctx.set_graphs(False)
    assert _same(ctx.sign_grad(eta, psi, 60, want_dpsi=True), ref60)
    ctx.close()


def test_graph_replays_match_eager_batched_colour_split():
    dims = (10, 10, 10, 10)
    r = np.random.default_rng(23)
    U = dev(random_links(dims, 0.4, r))
    ks = [20, 14, 17]
    psi = dev(np.stack([z2_complex_source(10000, r) for _ in ks]))
    eta = dev(np.stack([z2_complex_source(10000, r) for _ in ks]))
    torch.cuda.synchronize()
    ctx = _side_stream_ctx(dims, -2.0, 0.3, U)
    S0, dU0, _, _ = ctx.sign_grad_batched(eta, psi, ks)   # times the pair-kernel shape
    S1, dU1, _, _ = ctx.sign_grad_batched(eta, psi, ks)
    assert S1 == S0 and torch.equal(dU1, dU0)
    ctx.set_graphs(True)
    for rep in range(3):
        say(f"graph 10^4 batch ks={ks}, call {rep}")
        S, dU, _, _ = ctx.sign_grad_batched(eta, psi, ks)
        assert S == S0 and torch.equal(dU, dU0), rep
        _eager_noise(dU)
    ctx.close()


def test_graphs_need_a_stream():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import TslovError
    ctx = Context((2, 2, 2, 4), -2.0, 0.3)   # the null (default) stream
    if ctx.stream.cuda_stream != 0:
        pytest.skip("the current stream is not the null stream")
    with pytest.raises(TslovError):
        ctx.set_graphs(True)
    ctx.close()
