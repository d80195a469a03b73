"""The paper's block-matrix derivative (Theorem 1, eq. func_derivative_1) and its error
estimate (eq. bA_error_est) on the GPU against oracle.blockderiv.

TSL of size k on B = [[H, dH], [0, H]] for one link parameter U_nu(x) -> exp(itX) U_nu(x):
* from (0, psi): the upper half (the derivative) and the lower half (the sign)
  against the oracle at the 4^4 workload (k = 40) for an su(3) and a U(1) direction,
  on a spatial link in the bulk and on a temporal link across the antiperiodic
  boundary (where the folded boundary sign must reach the tangent), to 1e-10 or
  10 sigma; at the 8^4 workload (k = 100) for one direction;
* from a general source (x1, x2) against the oracle's block process;
* eps_B against the oracle's (two block processes, the second from the first result);
* the deflated block process (App. E) on 2^3x4 and 3^3x4 lattices with l = 10 and 20
  eigenpairs of the dense H: both halves from a general source (x1, x2) and from
  (0, psi), and the deflated eps_B, against oracle.blockderiv.deflated_block_sign
  (eigenvector derivatives from the full dense spectrum), to 1e-10.
"""
import numpy as np
import pytest

from gpu_util import dev, host, rel, say
from oracle import blockderiv as BD
from oracle import grad as GR
from oracle.wilson import WilsonOperator
from synthetic import config_rng, workload, z2_complex_source

pytestmark = pytest.mark.gpu


def _ctx(wl):
    from paper_1604_08057_amd import Context
    ctx = Context(wl.dims, wl.mass, wl.mu)
    ctx.set_links(dev(wl.links()))
    return ctx


def _cases(wl):
    r = config_rng(wl.config, 4)
    V3 = wl.dims[0] * wl.dims[1] * wl.dims[2]
    last_t = (wl.dims[3] - 1) * V3 + 5          # a site on the last time slice
    return [(0, 17, GR.su3_direction(r)), (3, last_t, GR.su3_direction(r)), (3, last_t, np.eye(3, dtype=complex)),
            (1, 40, np.eye(3, dtype=complex))]


@pytest.mark.parametrize("config,k", [(1, 40), (2, 100)])
def test_block_derivative_against_oracle(config, k):
    wl = workload(config)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi = wl.links(), wl.psi()
    ctx = _ctx(wl)
    cases = _cases(wl) if config == 1 else _cases(wl)[1:2]
    perm = np.random.default_rng(0).permutation(24 * op.volume)
    for nu, site, X in cases:
        ref = BD.d1_derivative(op, U, psi, k, nu, site, X)
        alt = BD.d1_derivative(op, U, psi, k, nu, site, X, perm=perm)
        sig = max(rel(alt["y1"], ref["y1"]), rel(alt["y2"], ref["y2"]))
        y1, y2, info = ctx.block_sign(nu, site, X, dev(psi), k)
        e1, e2 = rel(host(y1), ref["y1"]), rel(host(y2), ref["y2"])
        say(f"block derivative {wl.dims} k={k} link ({nu}, {site}): d/dt err {e1:.2e} sign err {e2:.2e} "
            f"(sigma {sig:.2e}) k_used {info.k_used} ms {info.ms[5]:.1f}")
        assert info.k_used == ref["k_used"]
        assert e1 < max(1e-10, 10 * sig) and e2 < max(1e-10, 10 * sig)
    ctx.close()


def test_block_process_general_source_and_error_estimate():
    wl = workload(1)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi = wl.links(), wl.psi()
    nu, site, X = _cases(wl)[1]
    x1 = z2_complex_source(wl.volume, np.random.default_rng(8))
    k = 30
    bop = BD.BlockOperator(op, U, BD.link_direction_field(U, nu, site, X), psi.shape)
    ref = BD.block_tsl(bop, x1, psi, k)
    ctx = _ctx(wl)
    y1, y2, info = ctx.block_sign(nu, site, X, dev(psi), k, x1=dev(x1))
    e1, e2 = rel(host(y1), ref["y1"]), rel(host(y2), ref["y2"])
    eps = ctx.block_error_estimate(nu, site, X, dev(psi), k)
    ctx.close()
    want = BD.eps_block(op, U, psi, k, nu, site, X)
    say(f"block process from (x1, x2), k={k}: errs {e1:.2e} {e2:.2e}; eps_B {eps:.10e} (oracle {want:.10e})")
    assert e1 < 1e-10 and e2 < 1e-10
    assert abs(eps - want) < 1e-9 * want


@pytest.mark.parametrize("dims,l,k", [((2, 2, 2, 4), 10, 24), ((3, 3, 3, 4), 20, 40)])
def test_deflated_block_process_against_oracle(dims, l, k):
    from paper_1604_08057_amd import Context
    from oracle import deflation as DF
    from oracle.wilson import dense_h
    from synthetic import random_links
    mass, mu = -2.0, 0.3
    r = np.random.default_rng(41)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, r)
    psi, x1 = z2_complex_source(V, r), z2_complex_source(V, r)
    nu, site, X = 3, V - 2, GR.su3_direction(r)
    op = WilsonOperator(dims, mass, mu)
    dU = BD.link_direction_field(U, nu, site, X)
    lam, R, L = DF.eigenpairs(dense_h(U, dims, mass, mu), l)
    ctx = Context(dims, mass, mu)
    ctx.set_links(dev(U))
    defl = ctx.deflation(dev(R.T.reshape(l, V, 4, 3)), dev(L.T.reshape(l, V, 4, 3)), lam)
    for src1 in (x1, None):
        ref = BD.deflated_block_sign(op, U, dU, np.zeros_like(psi) if src1 is None else src1, psi, k, l, dims, mass, mu)
        y1, y2, info = ctx.block_sign(nu, site, X, dev(psi), k, x1=None if src1 is None else dev(src1), defl=defl)
        e1, e2 = rel(host(y1), ref["y1"]), rel(host(y2), ref["y2"])
        say(f"deflated block process {dims} l={l} k={k} x1={'general' if src1 is not None else 'zero'}: "
            f"errs {e1:.2e} {e2:.2e}, CG iterations {info.cg_iters}")
        assert e1 < 1e-10 and e2 < 1e-10
    eps = ctx.block_error_estimate(nu, site, X, dev(psi), k, defl=defl)
    eps0 = ctx.block_error_estimate(nu, site, X, dev(psi), k)
    ctx.close()
    want = BD.eps_block_deflated(op, U, dU, psi, k, l, dims, mass, mu)
    say(f"  deflated eps_B {eps:.10e} (oracle {want:.10e}; undeflated {eps0:.3e})")
    assert abs(eps - want) < 1e-9 * want


def test_deflated_block_process_errors():
    """A deflated eigenvalue on the imaginary axis gives ERR_SIGN_UNDEFINED; a non-finite
    direction or a link out of range ERR_ARG; one eigenpair (l = 1) against the oracle;
    the operator form of the shifted solves must be 0..3."""
    from paper_1604_08057_amd import Context
    from paper_1604_08057_amd.tslov import ERR_ARG, ERR_SIGN_UNDEFINED, TslovError
    from oracle import deflation as DF
    from oracle.wilson import dense_h
    from synthetic import random_links
    dims, mass, mu = (2, 2, 2, 4), -2.0, 0.3
    r = np.random.default_rng(47)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, r)
    psi = z2_complex_source(V, r)
    lam, R, L = DF.eigenpairs(dense_h(U, dims, mass, mu), 1)
    ctx = Context(dims, mass, mu)
    ctx.set_links(dev(U))
    Rd, Ld = dev(R.T.reshape(1, V, 4, 3)), dev(L.T.reshape(1, V, 4, 3))
    X = GR.su3_direction(r)
    for bad in (np.array([0.0 + 0.2j]),):
        with pytest.raises(TslovError) as e:
            ctx.block_sign(1, 3, X, dev(psi), 16, defl=ctx.deflation(Rd, Ld, bad))
        assert e.value.status == ERR_SIGN_UNDEFINED
    defl = ctx.deflation(Rd, Ld, lam)
    for nu, site, Xb in ((4, 3, X), (1, V, X), (1, 3, np.full((3, 3), np.nan, dtype=complex))):
        with pytest.raises(TslovError) as e:
            ctx.block_sign(nu, site, Xb, dev(psi), 16, defl=defl)
        assert e.value.status == ERR_ARG
    for form in (-1, 4):
        with pytest.raises(TslovError) as e:
            ctx.set_cg_operator(form)
        assert e.value.status == ERR_ARG
    y1, y2, info = ctx.block_sign(1, 3, X, dev(psi), 16, defl=defl)
    ctx.close()
    op = WilsonOperator(dims, mass, mu)
    ref = BD.deflated_block_sign(op, U, BD.link_direction_field(U, 1, 3, X), np.zeros_like(psi), psi, 16, 1, dims,
                                 mass, mu)
    e1, e2 = rel(host(y1), ref["y1"]), rel(host(y2), ref["y2"])
    say(f"deflated block process, one eigenpair: errs {e1:.2e} {e2:.2e}, CG iterations {info.cg_iters}")
    assert e1 < 1e-10 and e2 < 1e-10
