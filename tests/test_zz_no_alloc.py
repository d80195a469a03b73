"""The allocation-free operator entry point (tslov_apply_h_noalloc) against
tslov_apply_h: the same bits, on two calls in a row whose second has a smaller
lattice (a second context on the same device, sharing the device's scratch
array), in float64, float32-link and float32 contexts, both daggers; and the
size limit."""
import numpy as np
import pytest
import torch

from gpu_util import dev, say
from synthetic import random_links, z2_complex_source

pytestmark = pytest.mark.gpu


def _pair(dims, precision, seed):
    from paper_1604_08057_amd import Context
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    ctx = Context(dims, -2.0, 0.3, precision=precision)
    ctx.set_links(dev(random_links(dims, 0.4, rng)))
    x = dev(z2_complex_source(V, rng))
    out = []
    for dagger in (False, True):
        want = ctx.apply_h(x, dagger=dagger)
        got = torch.full_like(want, float("nan"))
        ctx.apply_h_noalloc(x, got, dagger=dagger)
        torch.cuda.synchronize()
        out.append((want, got))
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32links", "mixed"])
def test_noalloc_operator_matches(precision):
    for dims, seed in (((16, 16, 16, 16), 1), ((6, 4, 8, 10), 2)):   # the second call is smaller
        say(f"noalloc operator {precision} dims={dims}")
        for want, got in _pair(dims, precision, seed):
            assert torch.equal(got, want)


def test_noalloc_size_limit():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import ERR_ARG, TslovError
    dims = (18, 18, 18, 16)            # 93312 sites: above the float64 limit of 87381
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(torch.zeros((4, 93312, 3, 3), dtype=torch.complex128, device="cuda")
                  + torch.eye(3, dtype=torch.complex128, device="cuda"))
    x = torch.zeros((93312, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(TslovError) as e:
        ctx.apply_h_noalloc(x, torch.empty_like(x))
    assert e.value.status == ERR_ARG
    ctx.close()
