"""GPU two-sided Lanczos sgn(H)psi and D_ov psi against the oracle TSL at the same k.

Bar: 1e-10 relative (2-norm) in FP64, the bound for same-k parity while the
oracle's own reduction-order sensitivity stays below 1e-11 (measured by the
oracle tests).  Cases: the 4^4 workload (k = 64), a ragged lattice, the 8^4
workload (k = 200), the lucky breakdown of a free-field plane wave (exact at
k = 2), k = 1, and the float32 path (error against FP64 reported, bounded).
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle import wilson as W
from synthetic import random_links, workload, z2_complex_source

pytestmark = pytest.mark.gpu


def _run(dims, mass, mu, U, psi, k, precision="fp64"):
    from paper_1604_08057_amd import Context
    ctx = Context(dims, mass, mu, precision=precision)
    ctx.set_links(dev(U))
    y, info = ctx.sign(dev(psi), k)
    d, _ = ctx.overlap(dev(psi), k)
    out = host(y), host(d), info
    ctx.close()
    return out


@pytest.mark.parametrize("config", [1, 2])
def test_sign_and_overlap_workloads(config):
    wl = workload(config)
    say(f"tsl workload {config} dims={wl.dims} k={wl.k}")
    U, psi = wl.links(), wl.psi()
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    ref = GR.forward(op, U, psi, wl.k)
    y, d, info = _run(wl.dims, wl.mass, wl.mu, U, psi, wl.k)
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    say(f"  k_used={info.k_used} newton={info.newton_iters} y err {rel(y, ref['y']):.2e} "
        f"ms={info.ms[5]:.1f}")
    assert info.k_used == ref["k_used"] == wl.k
    assert rel(y, ref["y"]) < 1e-10
    assert rel(d, psi + g5 * ref["y"]) < 1e-10


def test_ragged_lattice():
    dims = (3, 5, 7, 6)
    rng = np.random.default_rng(9)
    U = random_links(dims, 0.45, rng)
    psi = z2_complex_source(int(np.prod(dims)), rng)
    op = W.WilsonOperator(dims, -2.0, 0.25)
    ref = GR.forward(op, U, psi, 40)
    y, _, info = _run(dims, -2.0, 0.25, U, psi, 40)
    assert rel(y, ref["y"]) < 1e-10


def test_k_one():
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(2)
    U = random_links(dims, 0.5, rng)
    psi = z2_complex_source(256, rng)
    op = W.WilsonOperator(dims, -2.0, 0.3)
    ref = GR.forward(op, U, psi, 1)
    y, _, info = _run(dims, -2.0, 0.3, U, psi, 1)
    assert info.k_used == 1
    assert rel(y, ref["y"]) < 1e-13


def test_free_field_lucky_breakdown():
    dims = (4, 4, 4, 4)
    V = 256
    mass, mu = -1.5, 0.3
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    p = [2 * math.pi / 4, 0.0, 2 * math.pi * 2 / 4, math.pi * 3 / 4]
    chi = np.arange(12).reshape(4, 3) * (0.3 + 0.1j) + 1.0
    psi = W.plane_wave(dims, p, chi)
    y, _, info = _run(dims, mass, mu, U, psi, 20)
    h = W.gamma5() @ W.free_field_symbol(p, mass, mu)
    want = W.plane_wave(dims, p, (h / np.sqrt((h @ h)[0, 0])) @ chi)
    say(f"  free field k_used={info.k_used} breakdown={info.breakdown} err {np.abs(y - want).max():.2e}")
    assert info.k_used == 2 and info.breakdown == 1
    assert np.abs(y - want).max() < 1e-12


def test_mixed_precision_error_is_bounded():
    wl = workload(2)
    U, psi = wl.links(), wl.psi()
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    ref = GR.forward(op, U, psi, wl.k)
    y, _, info = _run(wl.dims, wl.mass, wl.mu, U, psi, wl.k, precision="mixed")
    err = rel(y, ref["y"])
    say(f"  mixed (float32 stencil and vectors) vs fp64 oracle, 8^4 k=200: {err:.2e}")
    assert err < 1e-3


def test_argument_errors():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import ERR_ARG, TslovError
    ctx = Context((4, 4, 4, 4), -2.0, 0.3)
    x = torch.zeros((256, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(TslovError) as e:
        ctx.sign(x, 8)                       # links not set
    assert e.value.status == ERR_ARG
    ctx.set_links(dev(random_links((4, 4, 4, 4), 0.5, np.random.default_rng(0))))
    with pytest.raises(TslovError) as e:
        ctx.sign(x + 1, 0)
    assert e.value.status == ERR_ARG
    with pytest.raises(TslovError) as e:
        ctx.sign(x + 1, 2000)
    assert e.value.status == ERR_ARG
    y = x + 1
    with pytest.raises(TslovError):
        ctx.sign(y, 4, out=y)                # in place not allowed
    ctx.close()
