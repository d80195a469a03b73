"""Differentiation with deflation at the 16^4 workload (Sec. 3, App. E, eq. final_res).

Field: the 16^4 workload's gauge-rotated constant SU(3) field (mass -2, mu = 0.3),
whose 20 eigenpairs of smallest |lambda| (|lambda| 0.033 ... 0.068, each at least
6.4e-3 from every other eigenvalue) come from oracle.constfield in closed form;
k = 400, one Z2 source psi and probe eta.

* eigenpairs: residuals of two pairs under the oracle's gather stencil (CPU);
* forward: the deflated sgn(H) psi at k = 400 against the exact sign (the
  closed-form spectral sign).  Its components along the deflated directions,
  L_i^H sgn(H) psi = s_i L_i^H psi, must be exact (the TSL part lives in the
  invariant complement), where the undeflated run misses them; the remaining
  error is the TSL error at this k (the field has eigenvalues near the imaginary
  axis away from zero), which eps_A must estimate within a factor 10;
* derivative of S = Re <eta|D_ov|psi> through SignGrad (deflated, Krylov vectors
  regenerated in segments of 20):
  - the U(1) Ward identity at every site, which holds only with the eigenpair
    motion included;
  - the directional derivative along C_nu -> exp(i t X) C_nu (nu = x and t), a
    direction that keeps the field solvable (every link moves), against
    Richardson-extrapolated central differences of the library forward, each side
    deflated by the exact eigenpairs of its own field, to 1e-6;
  - recompute = 20 against storing every Krylov vector (same S, dS/dU to 1e-12);
  - the FP32-link variant of the same derivative, error against FP64 stated;
* the four operator forms of the 40 shifted solves (multi-right-hand-side,
  colour split, matrix-core and t-march) give the same derivative to 1e-9 (each
  solve stops at relative residual 1e-13; the forms differ in the order of the
  residual-norm sums and, on the matrix cores, of the link products), with the
  time of each;
* two sources in one batched deflated call (80 shifted systems in one CGNR): the
  second equal bit for bit to its single-source call; the deflated current estimator
  over the two sources with its Ward residual below 1e-9.
"""
import numpy as np
import pytest
import torch
from scipy.linalg import expm

from gpu_util import dev, host, rel, say
from oracle import constfield as CF
from oracle import grad as GR
from oracle.wilson import WilsonOperator, gamma5
from synthetic import workload
from synthetic.fields import links_from_constant

pytestmark = pytest.mark.gpu

G5 = np.diag(gamma5()).real


@pytest.fixture(scope="module")
def c5():
    wl = workload(5)
    U, C, g = wl.constant_field()
    eig = CF.lowest_eigenpairs(wl.dims, wl.mass, wl.mu, C, g, wl.n_deflate)
    say(f"16^4 eigenpairs: |lambda| {abs(eig['lam'][0]):.4f} .. {abs(eig['lam'][-1]):.4f}, "
        f"min separation {eig['separation'].min():.2e}, edge {eig['edge']}")
    return dict(wl=wl, U=U, C=C, g=g, eig=eig, psi=wl.psi(), eta=wl.eta())


def _ctx(wl, U, precision="fp64"):
    from paper_1604_08057_amd import Context
    ctx = Context(wl.dims, wl.mass, wl.mu, precision=precision)
    ctx.set_links(dev(U))
    return ctx


def test_eigenpairs_under_gather_stencil(c5):
    wl, eig = c5["wl"], c5["eig"]
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    Ut = torch.from_numpy(c5["U"])
    for i in (0, wl.n_deflate - 1):
        r, q = torch.from_numpy(eig["R"][i]), torch.from_numpy(eig["L"][i])
        er = (op.h(Ut, r) - eig["lam"][i] * r).norm().item() / r.norm().item()
        el = (op.h_dag(Ut, q) - np.conj(eig["lam"][i]) * q).norm().item() / q.norm().item()
        say(f"  pair {i}: |H R - lam R| {er:.1e}, |H^dag L - conj(lam) L| {el:.1e}")
        assert er < 1e-13 and el < 1e-13


def test_deflated_overlap_against_exact(c5):
    wl, eig, psi = c5["wl"], c5["eig"], c5["psi"]
    exact = psi + G5[None, :, None] * CF.exact_sign(wl.dims, wl.mass, wl.mu, c5["C"], c5["g"], psi)
    ctx = _ctx(wl, c5["U"])
    defl = ctx.deflation(dev(eig["R"]), dev(eig["L"]), eig["lam"])
    yd, info = ctx.overlap(dev(psi), wl.k, defl=defl)
    yp, _ = ctx.overlap(dev(psi), wl.k)
    eps = ctx.error_estimate(dev(psi), wl.k, defl=defl)
    ctx.close()
    ed, ep = rel(host(yd), exact), rel(host(yp), exact)
    # the sign's error relative to |psi| (D_ov psi - psi = g5 sgn(H) psi)
    es = np.linalg.norm(host(yd) - exact) / np.linalg.norm(psi)
    Lf = eig["L"].reshape(wl.n_deflate, -1).conj()
    c = Lf @ psi.ravel()
    want = np.sign(eig["lam"].real) * c
    sgn = lambda y: (G5[None, :, None] * (host(y) - psi)).ravel()  # noqa: E731
    cd = np.abs(Lf @ sgn(yd) - want).max() / np.abs(c).max()
    cp = np.abs(Lf @ sgn(yp) - want).max() / np.abs(c).max()
    say(f"16^4 k={wl.k}: D_ov psi error deflated {ed:.2e} (sign {es:.2e}, eps_A {eps:.2e}), "
        f"undeflated {ep:.2e}; deflated components: deflated run {cd:.2e}, undeflated run {cp:.2e}; "
        f"k_used {info.k_used} ms {info.ms[5]:.1f}")
    assert info.k_used == wl.k
    assert cd < 1e-10 and cp > 1e3 * cd
    assert 0.1 * eps < es < 10 * eps


def _directional(G, U, g, nu, X):
    """sum_x Re tr(G_nu(x)^H i g(x) X g(x)^H U_nu(x))."""
    dU = 1j * np.einsum("vab,bc,vdc,vde->vae", g, X, g.conj(), U[nu])
    return float(np.real(np.einsum("vab,vab->", G[nu].conj(), dU)))


def test_deflated_derivative_ward_fd_recompute(c5):
    from paper_1604_08057_amd import SignGrad
    wl, eig, U, C, g = c5["wl"], c5["eig"], c5["U"], c5["C"], c5["g"]
    psi, eta = c5["psi"], c5["eta"]
    ctx = _ctx(wl, U)
    defl = ctx.deflation(dev(eig["R"]), dev(eig["L"]), eig["lam"])
    Ut = dev(U).requires_grad_(True)
    pt, et = dev(psi).requires_grad_(True), dev(eta).requires_grad_(True)
    S = SignGrad.apply(Ut, pt, et, ctx, wl.k, 20, defl, True)
    S.backward()
    G, dpsi, dov = host(Ut.grad), host(pt.grad), host(et.grad)
    say(f"16^4 deflated derivative (l=20, k={wl.k}, recompute 20): S {S.item():.12e}")

    lhs, rhs = GR.ward_residual(WilsonOperator(wl.dims, wl.mass, wl.mu), G, U, psi, eta, dov, dpsi)
    ward = np.abs(lhs - rhs).max() / np.abs(lhs).max()
    say(f"  Ward identity: max |lhs - rhs| / max |lhs| = {ward:.2e}")
    assert ward < 1e-9

    S0, dU0, dp0, dov0, info0 = ctx.overlap_grad(dev(eta), dev(psi), wl.k, defl=defl)
    eG, eP, eY = rel(G, host(dU0)), rel(dpsi, host(dp0)), rel(dov, host(dov0))
    say(f"  store-all vs recompute 20: S equal {S0 == S.item()}, dU {eG:.2e}, dpsi {eP:.2e}, D_ov psi {eY:.2e}, "
        f"CG iterations {info0.cg_iters}, ms {info0.ms[5]:.0f}")
    assert S0 == S.item() and eG < 1e-12 and eP < 1e-12 and eY < 1e-13

    rng = np.random.default_rng([1604, 8057, 5, 4])
    for nu in (0, 3):
        X = GR.su3_direction(rng)
        want = _directional(G, U, g, nu, X)
        fd = {}
        for h in (2e-4, 1e-4):
            vals = []
            for s in (1.0, -1.0):
                Ch = C.copy()
                Ch[nu] = expm(1j * s * h * X) @ C[nu]
                lam, R, L, jump = CF.tracked_eigenpairs(wl.dims, wl.mass, wl.mu, Ch, g, eig["labels"], eig["lam"])
                ctx.set_links(dev(links_from_constant(Ch, g, wl.dims)))
                d = ctx.deflation(dev(R), dev(L), lam)
                y, _ = ctx.overlap(dev(psi), wl.k, defl=d)
                vals.append(float(np.real(np.vdot(eta.ravel(), host(y).ravel()))))
            fd[h] = (vals[0] - vals[1]) / (2 * h)
        rich = (4 * fd[1e-4] - fd[2e-4]) / 3
        e = abs(rich - want) / abs(want)
        say(f"  direction C_{nu} -> exp(itX) C_{nu}: gradient {want:.10e}, FD {rich:.10e} "
            f"(h=2e-4 {fd[2e-4]:.10e}), rel err {e:.2e}")
        assert e < 1e-6
    ctx.set_links(dev(U))
    ctx.close()

    c32 = _ctx(wl, U, precision="fp32links")
    d32 = c32.deflation(dev(eig["R"]), dev(eig["L"]), eig["lam"])
    S32, dU32, dp32, dov32, i32 = c32.overlap_grad(dev(eta), dev(psi), wl.k, defl=d32, recompute=20)
    c32.close()
    say(f"  fp32 links vs fp64: S {abs(S32 - S0) / abs(S0):.2e}, dU {rel(host(dU32), host(dU0)):.2e}, "
        f"dpsi {rel(host(dp32), host(dp0)):.2e}, D_ov psi {rel(host(dov32), host(dov0)):.2e}")


def test_shifted_solve_operator_forms(c5):
    wl, eig, U = c5["wl"], c5["eig"], c5["U"]
    psi, eta = c5["psi"], c5["eta"]
    ctx = _ctx(wl, U)
    defl = ctx.deflation(dev(eig["R"]), dev(eig["L"]), eig["lam"])
    res = {}
    for form in (0, 1, 2, 3):
        ctx.set_cg_operator(form)
        S, dU, dp, dov, info = ctx.overlap_grad(dev(eta), dev(psi), wl.k, defl=defl, recompute=20)
        res[form] = (S, host(dU), host(dp), info)
        say(f"16^4 deflated derivative, operator form {form}: CG iterations {info.cg_iters}, "
            f"solves {info.ms[4]:.0f} ms, total {info.ms[5]:.0f} ms")
    ctx.close()
    S1, G1, P1, _ = res[1]
    for form in (0, 2, 3):
        S0, G0, P0, _ = res[form]
        eS, eG, eP = abs(S0 - S1) / abs(S1), rel(G0, G1), rel(P0, P1)
        say(f"  form {form} vs colour split: S {eS:.2e} dU {eG:.2e} dpsi {eP:.2e}")
        assert eS < 1e-12 and eG < 1e-9 and eP < 1e-9


def test_batched_deflated_derivative_and_current(c5):
    """Two sources of the 16^4 workload in one batched deflated call (80 shifted systems in
    one CGNR): the second equal bit for bit to its single-source call; the deflated
    current estimator over the same two Z2 sources has Ward residual below 1e-9."""
    wl, eig, U = c5["wl"], c5["eig"], c5["U"]
    psi, eta = c5["psi"], c5["eta"]
    ks = [wl.k, wl.k // 2]
    ctx = _ctx(wl, U)
    defl = ctx.deflation(dev(eig["R"]), dev(eig["L"]), eig["lam"])
    psis, etas = np.stack([psi, eta]), np.stack([eta, psi])
    S, dU, dpsi, infos = ctx.sign_grad_batched(dev(etas), dev(psis), ks, want_dpsi=True, defl=defl)
    S1, dU1, dp1, i1 = ctx.sign_grad(dev(etas[1]), dev(psis[1]), ks[1], want_dpsi=True, defl=defl)
    same = S1 == S[1] and torch.equal(dU1, dU[1]) and torch.equal(dp1, dpsi[1])
    say(f"16^4 batched deflated derivative, k={ks}: CG iterations {infos[0].cg_iters} (single {i1.cg_iters}), "
        f"{infos[0].ms[5]:.0f} ms for both vs {i1.ms[5]:.0f} ms for one; source 1 equal to single: {same}")
    assert same
    del dU, dpsi, dU1, dp1
    j, div, tot, ward, cinf = ctx.current_estimate(dev(psis), ks, defl=defl)
    ctx.close()
    say(f"  deflated current over 2 sources: Ward residual {ward:.2e}, max|div| / max|j| "
        f"{host(div).__abs__().max() / host(j).__abs__().max():.2e}")
    assert ward < 1e-9
