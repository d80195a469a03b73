"""GPU Wilson stencil against the oracle (App. A, eq. WD_op): D_w, D_w^dag, H, H^dag.

Lattices: 4^4, a ragged 3x5x7x6 (V = 630, not a multiple of the block size)
and 8^4 (colour-grid layout); 10^4 and a ragged 9x11x13x7 (V = 9009) above it
(site-per-thread operator, colour-split Lanczos kernels, XCD-padded grids);
16^3x32 and 32^3x8 (the t-march operator with the wrap in t, its chunk length
timed on the first call), where every forced chunk length (1, 2, 4, 8 slices)
gives the same bits; and the 32^4 lattice of the stencil benchmark (t-march)
with its own link and source generator.  FP64 is compared element by element to 1e-14 relative (max norm);
the float32 path to 2e-6.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel_max, say
from oracle.wilson import WilsonOperator
from synthetic import random_links

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-14), ("mixed", 2e-6)])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 7, 6), (8, 8, 8, 8), (10, 10, 10, 10), (9, 11, 13, 7),
                                  (16, 16, 16, 32)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_operators_match_oracle(dims, mu, precision, tol):
    from paper_1604_08057_amd import Context
    say(f"stencil dims={dims} mu={mu} precision={precision}")
    rng = np.random.default_rng(100 + sum(dims))
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, rng)
    x = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    op = WilsonOperator(dims, -2.0, mu)
    Ut, xt = torch.from_numpy(U), torch.from_numpy(x)
    ctx = Context(dims, -2.0, mu, precision=precision)
    ctx.set_links(dev(U))
    xd = dev(x)
    cases = [
        ("dw", ctx.apply_dw(xd), op.dw(Ut, xt)),
        ("dw_dag", ctx.apply_dw(xd, dagger=True), op.dw_dag(Ut, xt)),
        ("h", ctx.apply_h(xd), op.h(Ut, xt)),
        ("h_dag", ctx.apply_h(xd, dagger=True), op.h_dag(Ut, xt)),
    ]
    torch.cuda.synchronize()
    for name, got, want in cases:
        err = rel_max(host(got), want.numpy())
        say(f"  {name}: rel max err {err:.2e}")
        assert err < tol, name
    ctx.close()


def test_antiperiodic_flag_off():
    from paper_1604_08057_amd import Context
    dims = (4, 4, 4, 6)
    rng = np.random.default_rng(3)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, rng)
    x = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    op = WilsonOperator(dims, -1.0, 0.2, antiperiodic_t=False)
    ctx = Context(dims, -1.0, 0.2, antiperiodic_t=False)
    ctx.set_links(dev(U))
    got = host(ctx.apply_h(dev(x)))
    assert rel_max(got, op.h(torch.from_numpy(U), torch.from_numpy(x)).numpy()) < 1e-14
    ctx.close()


def test_benchmark_lattice_32():
    # the operator exactly as the stencil benchmark times it (links and source from
    # torch's generator on the device, not SU(3)), against the oracle on the host
    from paper_1604_08057_amd import Context
    dims = (32, 32, 32, 32)
    V = 32 ** 4
    g = torch.Generator(device="cuda").manual_seed(1604)
    U = torch.randn((4, V, 3, 3), dtype=torch.complex128, device="cuda", generator=g)
    x = torch.randn((V, 4, 3), dtype=torch.complex128, device="cuda", generator=g)
    say("stencil 32^4 (benchmark configuration)")
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(U)
    got = host(ctx.apply_h(x))
    ctx.close()
    want = WilsonOperator(dims, -2.0, 0.3).h(U.cpu(), x.cpu()).numpy()
    err = rel_max(got, want)
    say(f"  h: rel max err {err:.2e}")
    assert err < 1e-14


def test_tmarch_lattice_32x8():
    from paper_1604_08057_amd import Context
    dims = (32, 32, 32, 8)
    rng = np.random.default_rng(328)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, rng)
    x = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    op = WilsonOperator(dims, -2.0, 0.3)
    Ut, xt = torch.from_numpy(U), torch.from_numpy(x)
    say("stencil 32^3x8 (t-march, chunks of 4 slices)")
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(dev(U))
    xd = dev(x)
    cases = [("dw", ctx.apply_dw(xd), op.dw(Ut, xt)), ("h_dag", ctx.apply_h(xd, dagger=True), op.h_dag(Ut, xt))]
    torch.cuda.synchronize()
    ctx.close()
    for name, got, want in cases:
        err = rel_max(host(got), want.numpy())
        say(f"  {name}: rel max err {err:.2e}")
        assert err < 1e-14, name


def test_tmarch_chunk_lengths_identical():
    # every chunk length of the marching operator gives the same bits (the first
    # slice of a chunk forms its backward t-hop with the same arithmetic as the
    # carried one), and the timed pick is one of them
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import TslovError
    dims = (32, 32, 32, 8)
    rng = np.random.default_rng(329)
    V = int(np.prod(dims))
    U, x = dev(random_links(dims, 0.5, rng)), dev(rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3)))
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(U)
    outs = {}
    for T in (1, 2, 4, 8):
        say(f"stencil 32^3x8, chunk of {T} slices")
        ctx.set_apply_chunk(T)
        outs[T] = ctx.apply_h(x)
    with pytest.raises(TslovError):
        ctx.set_apply_chunk(3)
    ctx.close()
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(U)
    timed = ctx.apply_h(x)
    pick = ctx.apply_chunk()
    ctx.close()
    say(f"  timed pick: {pick} slices per chunk")
    assert pick in (1, 2, 4, 8)
    for T in (2, 4, 8):
        assert torch.equal(outs[T], outs[1]), T
    assert torch.equal(timed, outs[1])
