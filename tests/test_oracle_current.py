"""Pins of the oracle link-current estimator (Sec. 4, divergence of the U(1) vector current).

* the exact trace Re Tr(g5 d sgn(H)/dTheta) is divergence free at every site
  (gauge invariance), while its total current is not zero;
* the estimator built from per-source rank-1 Daleckii-Krein gradients equals the
  matrix form with A = (1/N) sum_s xi_s (g5 xi_s)^H (linearity; two code paths);
* with the full Krylov space (k = n, re-biorthogonalised) the TSL estimator
  equals the exact-sign estimator for the same noise;
* the divergence of the TSL estimator equals the mean of the per-sample Ward
  source terms (catches a sign or neighbour error in the projection or the
  divergence), and a planted sign error in one link direction breaks it;
* the deflated estimator with every eigenpair deflated (l = n) equals the exact-sign
  estimator for the same noise (Daleckii-Krein, matrix form), and with l < n its
  divergence equals the mean Ward source terms of the deflated samples;
* the physical current Tr(D_ov^{-1} dD_ov/dTheta) (eq. lat_vec_cur) equals
  Richardson-extrapolated central differences of log det D_ov (Jacobi's formula),
  its divergence vanishes at every site while the total current does not, and one
  noise sample's divergence equals i [chi(x)^H (D_ov xi)(x) - |xi(x)|^2] with
  chi = D_ov^{-H} xi.
"""
import numpy as np
import pytest

from oracle import current as CU
from oracle import grad as GR
from oracle.wilson import WilsonOperator
from synthetic import random_links, z2_complex_source

DIMS, MASS, MU = (2, 2, 2, 4), -2.0, 0.3


@pytest.fixture(scope="module")
def setup():
    r = np.random.default_rng(11)
    U = random_links(DIMS, 0.5, r)
    xis = np.stack([z2_complex_source(32, r) for _ in range(3)])
    return U, xis, WilsonOperator(DIMS, MASS, MU)


def test_exact_current_is_divergence_free(setup):
    U, xis, op = setup
    j = CU.exact_current(U, DIMS, MASS, MU)
    div, tot = CU.divergence(j, op)
    assert np.abs(div).max() < 1e-11 * np.abs(j).max()
    assert np.abs(tot).max() > 1e-3 * np.abs(j).max()


def test_estimator_rank_one_vs_matrix_form(setup):
    U, xis, op = setup
    per = [GR.u1_projection(GR.exact_gradient(U, xi, CU.g5_source(xi), DIMS, MASS, MU), U) for xi in xis]
    A = sum(np.outer(xi.ravel(), CU.g5_source(xi).ravel().conj()) for xi in xis) / len(xis)
    jm = CU.exact_current(U, DIMS, MASS, MU, A=A)
    assert np.abs(np.mean(per, axis=0) - jm).max() < 1e-11 * np.abs(jm).max()


def test_full_krylov_estimator_is_exact():
    dims = (2, 2, 2, 2)
    r = np.random.default_rng(12)
    U = random_links(dims, 0.3, r)
    xis = np.stack([z2_complex_source(16, r) for _ in range(2)])
    op = WilsonOperator(dims, -1.2, 0.2)
    j, _ = CU.current_tsl(op, U, xis, [192, 192], reorth=True)
    A = sum(np.outer(xi.ravel(), CU.g5_source(xi).ravel().conj()) for xi in xis) / len(xis)
    jx = CU.exact_current(U, dims, -1.2, 0.2, A=A)
    assert np.linalg.norm(j - jx) / np.linalg.norm(jx) < 1e-6


def test_divergence_equals_mean_ward_source_terms(setup):
    U, xis, op = setup
    ks = [20, 13, 31]
    j, per = CU.current_tsl(op, U, xis, ks)
    div, _ = CU.divergence(j, op)
    rhs = np.mean([GR.ward_residual(op, p["G"], U, xi, CU.g5_source(xi), p["y"], p["dpsi"])[1]
                   for p, xi in zip(per, xis)], axis=0)
    assert np.abs(div - rhs).max() < 1e-10 * np.abs(j).max()
    jb = j.copy()
    jb[2] = -jb[2]   # planted error: wrong sign of one direction's projection
    divb, _ = CU.divergence(jb, op)
    assert np.abs(divb - rhs).max() > 1e-3 * np.abs(j).max()


# ------------------------------------------------------------------- the physical current (eq. lat_vec_cur)

@pytest.fixture(scope="module")
def gapped():
    dims, m, mu = (2, 2, 2, 4), -1.0, 0.3
    U = random_links(dims, 0.3, np.random.default_rng(2))
    return dims, m, mu, U, WilsonOperator(dims, m, mu)


def test_physical_current_is_the_derivative_of_log_det(gapped):
    """j(x, nu) = d/dTheta log det D_ov (Jacobi's formula), central differences of the
    dense determinant with the Schur sign."""
    dims, m, mu, U, op = gapped
    j = CU.physical_current(U, dims, m, mu)

    def logdet(Uh):
        s, l = np.linalg.slogdet(CU.overlap_dense(Uh, dims, m, mu))
        return np.log(s) + l
    def central(nu, site, h):
        Up, Um = U.copy(), U.copy()
        Up[nu, site] *= np.exp(1j * h)
        Um[nu, site] *= np.exp(-1j * h)
        return (logdet(Up) - logdet(Um)) / (2 * h)
    for nu, site in ((0, 3), (3, 29), (2, 17)):
        fd = (4 * central(nu, site, 1e-3) - central(nu, site, 2e-3)) / 3   # Richardson
        assert abs(fd - j[nu, site]) < 1e-8 * abs(j[nu, site])


def test_physical_current_divergence_vanishes(gapped):
    """Gauge invariance of det D_ov: zero divergence at every site, nonzero total current."""
    dims, m, mu, U, op = gapped
    j = CU.physical_current(U, dims, m, mu)
    dr, tr = CU.divergence(j.real, op)
    di, ti = CU.divergence(j.imag, op)
    assert np.abs(dr).max() < 1e-12 and np.abs(di).max() < 1e-12
    assert np.abs(tr).max() > 0.1 and np.abs(ti).max() > 0.1


def test_physical_current_sample_ward_identity(gapped):
    """One noise sample xi, chi = D_ov^{-H} xi: the divergence of chi^H dD_ov/dTheta xi at x
    is i [chi(x)^H (D_ov xi)(x) - |xi(x)|^2] (local U(1) rotation of chi^H D_ov xi)."""
    dims, m, mu, U, op = gapped
    xi = z2_complex_source(op.volume, np.random.default_rng(4))
    js = CU.physical_current(U, dims, m, mu, xi[None])
    D = CU.overlap_dense(U, dims, m, mu)
    chi = np.linalg.solve(D.conj().T, xi.ravel()).reshape(xi.shape)
    Dxi = (D @ xi.ravel()).reshape(xi.shape)
    want = 1j * (np.einsum("vsa,vsa->v", chi.conj(), Dxi) - np.einsum("vsa,vsa->v", xi.conj(), xi))
    dr, _ = CU.divergence(js.real, op)
    di, _ = CU.divergence(js.imag, op)
    assert np.abs(dr + 1j * di - want).max() < 1e-11 * np.abs(want).max()


def test_deflated_estimator_full_deflation_is_exact(setup):
    U, xis, op = setup
    n = 12 * op.volume
    j = CU.current_deflated(U, xis[:2], [8, 8], DIMS, MASS, MU, n)
    A = sum(np.outer(xi.ravel(), CU.g5_source(xi).ravel().conj()) for xi in xis[:2]) / 2
    jx = CU.exact_current(U, DIMS, MASS, MU, A=A)
    assert np.abs(j - jx).max() < 1e-9 * np.abs(jx).max()


def test_deflated_estimator_divergence_is_the_ward_source(setup):
    """sum_nu [j(x, nu) - j(x - nu, nu)] = mean over samples of -Im eta^H y + Im psibar^H psi
    at every site, y the deflated sign of xi and psibar its source gradient."""
    from oracle import deflation as DF
    from oracle.wilson import dense_h
    U, xis, op = setup
    l, k = 10, 12
    j = CU.current_deflated(U, xis[:2], [k, k], DIMS, MASS, MU, l)
    div, _ = CU.divergence(j, op)
    H = dense_h(U, DIMS, MASS, MU)
    lam, R, L = DF.eigenpairs(H, l)
    rhs = np.zeros(op.volume)
    for xi in xis[:2]:
        eta = CU.g5_source(xi)
        y = DF.deflated_sign(op, U, xi, k, lam, R, L)
        _, _, pb = DF.deflated_gradient(U, xi, eta, k, DIMS, MASS, MU, l)
        rhs += (-np.einsum("vab,vab->v", eta.conj(), y).imag + np.einsum("vab,vab->v", pb.conj(), xi).imag)
    rhs /= 2
    assert np.abs(div - rhs).max() < 1e-9 * np.abs(j).max()
