"""Per-call diagnostics and failure paths of the C ABI against the oracle.

* Ritz values: min |Re theta| and the norm of T_k against LAPACK on the oracle's
  own T_k (4^4, k = 64; 8^4, k = 200);
* biorthogonality probe |w_1^H v_k| + |w_k^H v_1| against the oracle's Lanczos
  vectors (its size, not its digits, is what rounding leaves alone: compared to
  a factor where it is above 1e-6, and both below 1e-6 otherwise);
* eps_A requested per call equals tslov_error_estimate's and the oracle's
  (Sec. 4.1 eq. error_est);
* the small dense step alone (tslov_tridiag_sign) against the oracle's Schur
  sign, and a constructed T with eigenvalues +-i: ERR_SIGN_UNDEFINED;
* a source that is an exact eigenvector of H (dense eigensolver of the oracle on
  a 2^3 x 4 lattice): lucky breakdown at j = 1 and the output sgn(Re lambda) psi;
* a non-finite link or source: ERR_ARG, and the context refuses to run on
  links it rejected;
* y_out of the derivative calls equals tslov_sign's output to rounding (their
  Newton iterations differ by one step) and bit for bit between the single and
  the batched derivative; the overlap derivative against the sign derivative and
  the oracle; the autograd function's eta gradient is the output.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle import wilson as W
from oracle.deflation import eigenpairs, error_estimate
from oracle.sign import sign_schur
from synthetic import random_links, workload, z2_complex_source

pytestmark = pytest.mark.gpu


def _ctx(wl, precision="fp64"):
    from paper_1604_08057_amd import Context
    ctx = Context(wl.dims, wl.mass, wl.mu, precision=precision)
    ctx.set_links(dev(wl.links()))
    return ctx


@pytest.mark.parametrize("config", [1, 2])
def test_ritz_and_biorthogonality(config):
    wl = workload(config)
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    ref = GR.forward(op, wl.links(), wl.psi(), wl.k)
    th = np.linalg.eigvals(ref["T"])
    ctx = _ctx(wl)
    _, info = ctx.sign(dev(wl.psi()), wl.k)
    ctx.close()
    nT = np.abs(ref["T"]).sum(axis=1).max()
    say(f"info workload {config}: min|Re theta| {info.min_abs_re_ritz:.6e} (oracle {np.abs(th.real).min():.6e}) "
        f"norm_T {info.norm_T:.4f} ({nT:.4f}) biorth {info.biorth_err:.3e} (oracle {ref['biorth']:.3e}) "
        f"flags {info.flags}")
    assert abs(info.min_abs_re_ritz - np.abs(th.real).min()) < 1e-9 * np.abs(th).max()
    assert abs(info.norm_T - nT) < 1e-10 * nT
    assert info.flags == 0
    if ref["biorth"] > 1e-6:
        assert 0.5 < info.biorth_err / ref["biorth"] < 2.0
    else:
        assert info.biorth_err < 1e-6


def test_eps_a_diagnostic():
    from paper_1604_08057_amd.tslov import DIAG_EPS_A
    wl = workload(1)
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi(), wl.eta()
    sign_fn = lambda x: GR.forward(op, U, x, wl.k)["y"]  # noqa: E731
    want = error_estimate(sign_fn, psi)
    ctx = _ctx(wl)
    e0 = ctx.error_estimate(dev(psi), wl.k)
    _, i_plain = ctx.sign(dev(psi), wl.k)
    ctx.set_diagnostics(DIAG_EPS_A)
    _, i_sign = ctx.sign(dev(psi), wl.k)
    _, i_ov = ctx.overlap(dev(psi), wl.k)
    *_, i_grad = ctx.sign_grad(dev(eta), dev(psi), wl.k)
    ctx.close()
    say(f"eps_A 4^4 k=64: oracle {want:.10e} estimate {e0:.10e} sign {i_sign.eps_A:.10e} "
        f"overlap {i_ov.eps_A:.10e} grad {i_grad.eps_A:.10e}")
    assert math.isnan(i_plain.eps_A)
    assert abs(e0 - want) < 1e-10 * want
    assert i_sign.eps_A == e0 and i_ov.eps_A == e0
    assert abs(i_grad.eps_A - e0) < 1e-10 * e0   # its y is the derivative's (see below)


def _tridiag(T):
    return np.diag(T).copy(), np.diag(T, -1).real.copy(), np.diag(T, 1).copy()


def test_tridiag_sign_and_sign_on_the_axis():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import ERR_SIGN_UNDEFINED, TslovError
    wl = workload(1)
    T = GR.forward(W.WilsonOperator(wl.dims, wl.mass, wl.mu), wl.links(), wl.psi(), wl.k)["T"]
    ctx = Context(wl.dims, wl.mass, wl.mu)
    c, info = ctx.tridiag_sign(*_tridiag(T))
    want = sign_schur(T)[:, 0]
    say(f"tridiag sign k={T.shape[0]}: err {rel(host(c), want):.2e} newton {info.newton_iters}")
    assert rel(host(c), want) < 1e-12
    # eigenvalues +-i (a 2x2 rotation block) beside a gapped remainder
    d = np.array([0.0, 0.0, 2.0, -1.5, 1.0, -2.5], dtype=np.complex128)
    sub = np.array([1.0, 0.0, 0.7, 0.4, 0.3])
    sup = np.array([-1.0, 0.0, 0.2 + 0.1j, -0.3j, 0.5], dtype=np.complex128)
    Tax = np.diag(d) + np.diag(sub, -1) + np.diag(sup, 1)
    assert np.abs(np.linalg.eigvals(Tax).real).min() < 1e-14
    with pytest.raises(TslovError) as e:
        ctx.tridiag_sign(d, sub, sup)
    say(f"  +-i block: {e.value}")
    assert e.value.status == ERR_SIGN_UNDEFINED
    ctx.close()


def test_eigenvector_source_stops_at_one_step():
    from paper_1604_08057_amd import Context
    dims = (2, 2, 2, 4)
    rng = np.random.default_rng(31)
    U = random_links(dims, 0.5, rng)
    H = W.dense_h(U, dims, -2.0, 0.3)
    lam, R, _ = eigenpairs(H, 3)
    ctx = Context(dims, -2.0, 0.3)
    ctx.set_links(dev(U))
    for i in range(3):
        psi = (R[:, i] / np.linalg.norm(R[:, i])).reshape(32, 4, 3)
        y, info = ctx.sign(dev(psi), 20)
        want = np.sign(lam[i].real) * psi
        say(f"eigenvector source lambda={lam[i]:.4f}: k_used {info.k_used} breakdown {info.breakdown} "
            f"err {rel(host(y), want):.2e}")
        assert info.k_used == 1 and info.breakdown == 1
        assert rel(host(y), want) < 1e-10
    ctx.close()


def test_non_finite_inputs():
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import ERR_ARG, TslovError
    wl = workload(1)
    ctx = Context(wl.dims, wl.mass, wl.mu)
    U = wl.links()
    U[2, 17, 1, 2] = np.nan
    with pytest.raises(TslovError) as e:
        ctx.set_links(dev(U))
    assert e.value.status == ERR_ARG and "non-finite" in str(e.value)
    with pytest.raises(TslovError) as e:
        ctx.sign(dev(wl.psi()), 8)          # the rejected links are not used
    assert e.value.status == ERR_ARG
    ctx.set_links(dev(wl.links()))
    psi = wl.psi()
    psi[5, 1, 0] = np.inf
    with pytest.raises(TslovError) as e:
        ctx.sign(dev(psi), 8)
    assert e.value.status == ERR_ARG
    y, info = ctx.sign(dev(wl.psi()), 8)    # the context still works
    assert info.k_used == 8
    ctx.close()


def test_y_out_equals_sign_output():
    # the derivative's Newton iteration takes one step more than the sign's (for the
    # Frechet block), so its y agrees with tslov_sign's to rounding, and bit for bit
    # between the single and the batched derivative calls
    wl = workload(1)
    ctx = _ctx(wl)
    y_sign, _ = ctx.sign(dev(wl.psi()), wl.k)
    S, _, _, info, y = ctx.sign_grad(dev(wl.eta()), dev(wl.psi()), wl.k, want_y=True)
    assert rel(host(y), host(y_sign)) < 1e-13
    psis = np.stack([wl.psi(), z2_complex_source(wl.volume, np.random.default_rng(4))])
    etas = np.stack([wl.eta(), wl.eta()])
    Sb, _, _, _, yb = ctx.sign_grad_batched(dev(etas), dev(psis), [wl.k, 40], want_y=True)
    y1, _ = ctx.sign(dev(psis[1]), 40)
    ctx.close()
    assert torch.equal(yb[0], y) and rel(host(yb[1]), host(y1)) < 1e-13
    assert Sb[0] == S
    assert abs(S - np.real(np.vdot(wl.eta(), host(y)))) < 1e-12 * abs(S)


def test_overlap_derivative_and_eta_gradient():
    from paper_1604_08057_amd import SignGrad
    wl = workload(1)
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi, eta = wl.links(), wl.psi(), wl.eta()
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    ctx = _ctx(wl)
    S, dU, dpsi, dov, _ = ctx.overlap_grad(dev(eta), dev(psi), wl.k)
    ref = GR.grad_autograd(op, U, psi, g5 * eta, wl.k)
    S_want = ref["S"] + np.real(np.vdot(eta, psi))
    say(f"overlap derivative: S err {abs(S - S_want) / abs(S_want):.2e} dU {rel(host(dU), ref['G']):.2e} "
        f"dpsi {rel(host(dpsi), eta + ref['dpsi']):.2e} D_ov psi {rel(host(dov), psi + g5 * ref['y']):.2e}")
    assert abs(S - S_want) < 1e-10 * abs(S_want)
    assert rel(host(dU), ref["G"]) < 1e-10
    assert rel(host(dpsi), eta + ref["dpsi"]) < 1e-10
    assert rel(host(dov), psi + g5 * ref["y"]) < 1e-10
    # through the autograd function: the eta gradient is D_ov psi (overlap) or y (sign)
    for overlap in (False, True):
        Ut = dev(U).requires_grad_(True)
        pt = dev(psi).requires_grad_(True)
        et = dev(eta).requires_grad_(True)
        St = SignGrad.apply(Ut, pt, et, ctx, wl.k, 0, None, overlap)
        (2.0 * St).backward()
        want_eta = (psi + g5 * ref["y"]) if overlap else GR.forward(op, U, psi, wl.k)["y"]
        assert rel(host(et.grad), 2.0 * want_eta) < 1e-10
        if overlap:
            assert rel(host(Ut.grad), 2.0 * ref["G"]) < 1e-10
            assert rel(host(pt.grad), 2.0 * (eta + ref["dpsi"])) < 1e-10
    ctx.close()
