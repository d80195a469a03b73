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
* 14x14^3 (V = 38416): sgn(H)psi at k = 100 against the oracle.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle.wilson import WilsonOperator
from synthetic import workload

pytestmark = pytest.mark.gpu


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
