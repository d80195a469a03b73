"""Nested projected-matrix step (one level of nesting, Sec. 4.1) against the oracle.

The GPU sign with tslov_set_nested(m) against oracle.nested (the same reading:
inner two-sided Lanczos of size m on (T_k^2)^{-1} from e_1, principal square root
of the inner matrix) at the same outer and inner sizes, on the 4^4 workload
(k = 64, m = 16, 32, 48) and the 8^4 workload (k = 200, m = 100), to 1e-10
relative or 10 sigma (sigma the oracle's own change when its outer inner products
are summed in a permuted order); an inner size at least k_used gives the plain
result bit for bit; the nested result approaches the plain one as m grows.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle import nested as N
from oracle.wilson import WilsonOperator
from synthetic import workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("config,m", [(1, 16), (1, 32), (1, 48), (2, 100)])
def test_nested_sign_against_oracle(config, m):
    from paper_1604_08057_amd import Context
    wl = workload(config)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi = wl.links(), wl.psi()
    ref = N.nested_tsl_wilson(op, U, psi, wl.k, m)
    perm = np.random.default_rng(0).permutation(12 * op.volume)
    alt = N.nested_tsl_wilson(op, U, psi, wl.k, m, perm=perm)
    sig = rel(alt["y"], ref["y"])
    plain = GR.forward(op, U, psi, wl.k)["y"]
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(U))
    ctx.set_nested(m)
    y, info = ctx.sign(dev(psi), wl.k)
    d, _ = ctx.overlap(dev(psi), wl.k)
    ctx.close()
    e = rel(host(y), ref["y"])
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    say(f"nested k={wl.k} m={m}: y err {e:.2e} (sigma {sig:.2e}) vs plain {rel(ref['y'], plain):.2e} "
        f"dense ms {info.ms[1]:.2f}")
    assert info.k_used == ref["k_used"]
    assert e < max(1e-10, 10 * sig)
    assert rel(host(d), psi + g5 * ref["y"]) < max(1e-10, 10 * sig)


def test_full_inner_size_is_plain():
    from paper_1604_08057_amd import Context
    wl = workload(1)
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(wl.links()))
    y0, _ = ctx.sign(dev(wl.psi()), wl.k)
    ctx.set_nested(wl.k)
    y1, _ = ctx.sign(dev(wl.psi()), wl.k)
    ctx.set_nested(0)
    ctx.close()
    assert torch.equal(y0, y1)
