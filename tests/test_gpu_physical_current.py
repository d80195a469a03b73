"""The physical U(1) vector current (Sec. 4.3 eq. lat_vec_cur, eq. divergence_def) on the GPU.

Workload: 3x4^3 (the size of the paper's check, mu = 0.3), smooth links and mass -1,
where the TSL sign has converged at k = 240 (eps_A 1.4e-13), so that D_ov with the
approximate sign is linear to that accuracy and can be inverted.  Against the
oracle's dense references (tests/golden/physical_current_3x4x4x4.npz, written by
make_current_refs.py from oracle/ alone):
* the overlap solves D_ov^{-1} b and D_ov^{-dag} b, to 1e-10;
* the estimator (1/N) sum_s chi_s^dag dD_ov/dTheta xi_s over the 4 Z2 sources
  against the same estimator with the exact operators, to 1e-9;
* its divergence at every site against the per-sample Ward identity,
  div = (1/N) sum_s i [chi_s(x)^dag (D_ov xi_s)(x) - |xi_s(x)|^2], built from the
  library's own solves and overlap applications, to 1e-9;
* the exact trace's divergence (oracle) vanishes while the estimator's total current
  does not (reported).
"""
import os

import numpy as np
import pytest

from gpu_util import dev, host, rel, say
from oracle import current as CU
from oracle.wilson import WilsonOperator
from synthetic import workload

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "physical_current_3x4x4x4.npz")


@pytest.fixture(scope="module")
def setup():
    from paper_1604_08057_amd import Context
    wl = workload(6)
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(wl.links()))
    yield wl, ctx, np.load(GOLD)
    ctx.close()


def test_overlap_solve(setup):
    wl, ctx, ref = setup
    b = dev(wl.psi()[0])
    for adj, key in ((False, "x"), (True, "x_adj")):
        x, it, rr = ctx.overlap_solve(b, wl.k, adjoint=adj, tol=1e-12)
        e = rel(host(x), ref[key])
        say(f"overlap solve 3x4^3 k={wl.k} adjoint={adj}: {it} iterations, residual {rr:.2e}, error {e:.2e}")
        assert e < 1e-10


def test_physical_current_estimator(setup):
    wl, ctx, ref = setup
    xis = wl.psi()
    res = ctx.physical_current(dev(xis), wl.k, tol=1e-12)
    j = host(res["j"])
    e = rel(j, ref["j_est"])
    say(f"physical current 3x4^3 k={wl.k}, {len(xis)} sources: error vs oracle estimator {e:.2e}; "
        f"solves {res['iters']} iterations; |j_est - j_exact| / |j_exact| = "
        f"{rel(ref['j_est'], ref['j_exact']):.2e}")
    assert e < 1e-9
    # per-sample Ward identity of the estimator, from the library's own solves and applications
    pred = np.zeros(wl.volume, dtype=np.complex128)
    for xi in xis:
        chi, _, _ = ctx.overlap_solve(dev(xi), wl.k, adjoint=True, tol=1e-12)
        dxi, _ = ctx.overlap(dev(xi), wl.k)
        pred += 1j * (np.einsum("vsa,vsa->v", host(chi).conj(), host(dxi)) - np.einsum("vsa,vsa->v", xi.conj(), xi))
    pred /= len(xis)
    div, tot = host(res["div"]), host(res["tot"])
    ew = np.abs(div - pred).max() / np.abs(pred).max()
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    dr, _ = CU.divergence(ref["j_exact"].real, op)
    di, _ = CU.divergence(ref["j_exact"].imag, op)
    say(f"  divergence vs per-sample Ward identity {ew:.2e}; estimator max |div| {np.abs(div).max():.3e}, "
        f"max |tot| {np.abs(tot).max():.3e}; exact trace max |div| {np.abs(dr + 1j * di).max():.1e}")
    assert ew < 1e-9
    assert np.abs(tot).max() > 0.1


def test_error_paths(setup):
    """A solve stopped before its tolerance returns ERR_NOT_CONVERGED (forced from the host
    with maxit = 1); bad tolerances and iteration limits are argument errors."""
    from paper_1604_08057_amd.tslov import ERR_ARG, ERR_NOT_CONVERGED, TslovError
    wl, ctx, _ = setup
    b = dev(wl.psi()[0])
    with pytest.raises(TslovError) as e:
        ctx.overlap_solve(b, wl.k, tol=1e-14, maxit=1)
    assert e.value.status == ERR_NOT_CONVERGED
    for kw in ({"tol": 0.0}, {"maxit": 0}):
        with pytest.raises(TslovError) as e:
            ctx.overlap_solve(b, wl.k, **kw)
        assert e.value.status == ERR_ARG
    with pytest.raises(TslovError) as e:
        ctx.physical_current(dev(wl.psi()), wl.k, tol=-1.0)
    assert e.value.status == ERR_ARG
