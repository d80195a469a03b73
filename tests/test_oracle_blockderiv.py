"""Pins of the oracle block-matrix derivative (the paper's method: Sec. 2 Theorem 1 and
eq. func_derivative_1; Sec. 3 Theorem 2 and the spectrum of B; Sec. 4.1 eq. bA_error_est).

* the projected matrix of TSL on B from (0, psi) is T_k of TSL on H from psi, and
  the lower half of the result is the sign itself;
* the upper half equals d/dt p(H + t dH) psi for the polynomial p that
  interpolates sgn at the Ritz values, evaluated in Newton form on the dense
  matrices of the independent dense builder (no Lanczos vectors);
* dH from the gauge field with one link i X U is the directional derivative of H:
  central differences of the dense H along exp(i t X) U;
* the spectrum of B is that of A, each eigenvalue twice (det B = det(A)^2), on a
  dense random example;
* Theorem 2: with d lambda_i != 0 every eigenvalue of B has one eigenvector and a
  2 x 2 Jordan block (rank of B - lambda and (B - lambda)^2); with dA a commutator
  [A, C] (all d lambda_i = 0) B is diagonalisable;
* eq. bA_error_est2 for a fixed block-triangular approximation
  [[S, dS], [0, S]]: the squared error splits into |S^2 psi - psi|^2 and
  |{S, dS} psi|^2, and vanishes for the exact sign and its Frechet derivative;
* eps_B of the TSL approximation falls with k on a gapped operator and stays
  within a factor of the true error of the derivative.
"""
import numpy as np
import scipy.linalg as sla
import torch

from oracle import blockderiv as BD
from oracle import grad as GR
from oracle import sign as SG
from oracle import wilson as W
from synthetic import random_links, z2_complex_source


def _problem(dims=(2, 2, 2, 4), spread=0.5, mass=-2.0, mu=0.3, seed=11):
    rng = np.random.default_rng(seed)
    U = random_links(dims, spread, rng)
    V = int(np.prod(dims))
    psi = z2_complex_source(V, rng)
    nu, site = 3, 5
    X = GR.su3_direction(rng)
    return dims, mass, mu, U, psi, nu, site, X


def test_block_process_reuses_the_plain_projected_matrix():
    dims, mass, mu, U, psi, nu, site, X = _problem()
    op = W.WilsonOperator(dims, mass, mu)
    k = 24
    d1 = BD.d1_derivative(op, U, psi, k, nu, site, X)
    plain = GR.forward(op, U, psi, k)
    assert d1["k_used"] == plain["k_used"] == k
    assert np.abs(d1["T"] - plain["T"]).max() < 1e-12 * np.abs(plain["T"]).max()
    assert np.linalg.norm(d1["y2"] - plain["y"]) < 1e-12 * np.linalg.norm(plain["y"])


def test_upper_half_is_the_frozen_polynomial_derivative():
    dims, mass, mu, U, psi, nu, site, X = _problem()
    op = W.WilsonOperator(dims, mass, mu)
    k = 24
    d1 = BD.d1_derivative(op, U, psi, k, nu, site, X)
    H = W.dense_h(U, dims, mass, mu)
    dH = W.dense_h(BD.link_direction_field(U, nu, site, X), dims, mass, mu) - W.dense_h(
        np.zeros_like(U), dims, mass, mu)
    ritz = np.linalg.eigvals(d1["T"])
    want = BD.frozen_polynomial_derivative(H, dH, psi.ravel(), ritz)
    got = d1["y1"].ravel()
    assert np.linalg.norm(got - want) < 1e-9 * np.linalg.norm(want)


def test_link_tangent_is_the_directional_derivative():
    dims, mass, mu, U, psi, nu, site, X = _problem()
    dH = W.dense_h(BD.link_direction_field(U, nu, site, X), dims, mass, mu) - W.dense_h(
        np.zeros_like(U), dims, mass, mu)
    h = 1e-5
    fd = (W.dense_h(GR.rotate_link(U, nu, site, X, h), dims, mass, mu)
          - W.dense_h(GR.rotate_link(U, nu, site, X, -h), dims, mass, mu)) / (2 * h)
    assert np.abs(fd - dH).max() < 1e-9


def _dense_pair(n, rng):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A, E


def test_spectrum_of_the_block_matrix():
    rng = np.random.default_rng(3)
    A, E = _dense_pair(8, rng)
    B = np.block([[A, E], [np.zeros_like(A), A]])
    eb = np.sort_complex(np.linalg.eigvals(B))
    ea = np.sort_complex(np.repeat(np.linalg.eigvals(A), 2))
    assert np.abs(eb - ea).max() < 1e-6      # double eigenvalues: perturbation ~ sqrt(eps)
    assert abs(np.linalg.det(B) - np.linalg.det(A) ** 2) < 1e-10 * abs(np.linalg.det(A)) ** 2


def test_theorem_2_jordan_structure():
    rng = np.random.default_rng(4)
    n = 6
    A, E = _dense_pair(n, rng)
    lam = np.linalg.eigvals(A)
    B = np.block([[A, E], [np.zeros_like(A), A]])
    scale = np.linalg.norm(B, 2)
    for li in lam:
        s1 = np.linalg.svd(B - li * np.eye(2 * n), compute_uv=False)
        s2 = np.linalg.svd((B - li * np.eye(2 * n)) @ (B - li * np.eye(2 * n)), compute_uv=False)
        assert s1[-1] < 1e-10 * scale and s1[-2] > 1e-6 * scale        # one eigenvector
        assert s2[-2] < 1e-9 * scale ** 2 and s2[-3] > 1e-6 * scale ** 2  # a 2 x 2 Jordan block
    C = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Bc = np.block([[A, A @ C - C @ A], [np.zeros_like(A), A]])         # d lambda_i = 0
    for li in lam:
        s = np.linalg.svd(Bc - li * np.eye(2 * n), compute_uv=False)
        assert s[-2] < 1e-9 * scale                                      # two eigenvectors


def test_block_error_estimate_identity():
    rng = np.random.default_rng(6)
    n = 10
    w = rng.uniform(0.3, 2.0, n) * rng.choice([-1, 1], n) + 0.3j * rng.standard_normal(n)
    Xm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = Xm @ np.diag(w) @ np.linalg.inv(Xm)
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    S, dS = SG.sign_schur(A), SG.frechet_sign(A, E)
    for pert in (0.0, 1e-3):
        Sp = S + pert * rng.standard_normal((n, n))
        dSp = dS + pert * rng.standard_normal((n, n))
        M = np.block([[Sp, dSp], [np.zeros_like(Sp), Sp]])
        z = np.concatenate([np.zeros(n), psi])
        lhs = np.linalg.norm(M @ (M @ z) - z) / (2 * np.linalg.norm(psi))
        rhs = np.hypot(np.linalg.norm(Sp @ Sp @ psi - psi), np.linalg.norm((Sp @ dSp + dSp @ Sp) @ psi)) / (
            2 * np.linalg.norm(psi))
        assert abs(lhs - rhs) < 1e-12 * max(rhs, 1e-300) + 1e-15
        if pert == 0.0:
            assert lhs < 1e-12


def test_block_error_estimate_tracks_the_derivative_error():
    dims, _, mu, U, psi, nu, site, X = _problem(spread=0.2, mass=-1.2, seed=12)
    mass = -1.2
    op = W.WilsonOperator(dims, mass, mu)
    H = W.dense_h(U, dims, mass, mu)
    dH = W.dense_h(BD.link_direction_field(U, nu, site, X), dims, mass, mu) - W.dense_h(
        np.zeros_like(U), dims, mass, mu)
    exact = SG.frechet_sign(H, dH) @ psi.ravel()
    errs, eps = [], []
    for k in (8, 16, 32):
        d1 = BD.d1_derivative(op, U, psi, k, nu, site, X)
        errs.append(np.linalg.norm(d1["y1"].ravel() - exact) / np.linalg.norm(psi))
        eps.append(BD.eps_block(op, U, psi, k, nu, site, X))
    assert all(b < a for a, b in zip(eps, eps[1:])), eps
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    for e, p in zip(errs, eps):
        assert 0.01 < p / e < 100.0, (errs, eps)


# ------------------------------------------------------------------ App. E deflation

def _defl_problem(l=12, seed=21):
    dims, mass, mu, U, psi, nu, site, X = _problem(seed=seed)
    rng = np.random.default_rng(seed + 1)
    op = W.WilsonOperator(dims, mass, mu)
    dU = BD.link_direction_field(U, nu, site, X)
    x1 = psi * 0.3 + 0.2 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    return dims, mass, mu, U, dU, op, x1, psi


def test_eigenvector_derivatives_match_finite_differences():
    """dR_i and <dL_i|x> (normalised <L_i|dR_i> = <dL_i|R_i> = 0) against central
    differences of the dense eigenvectors of H + t dH, each moved eigenvector scaled so
    that its overlap with the unmoved partner is 1."""
    dims, mass, mu, U, dU, op, x1, psi = _defl_problem()
    H = W.dense_h(U, dims, mass, mu)
    dH = W.dense_h(U + dU, dims, mass, mu) - H
    l = 6
    lam, R, L, dR, dLx = BD.eigenvector_derivatives(H, dH, l)
    x = x1.ravel()
    h = 1e-6
    moved = {}
    for s in (1.0, -1.0):
        w, vl, vr = sla.eig(H + s * h * dH, left=True, right=True)
        moved[s] = (w, vl, vr)
    dLx_want = np.zeros(l, dtype=np.complex128)
    for i in range(l):
        cols = {}
        for s, (w, vl, vr) in moved.items():
            j = int(np.argmin(np.abs(w - lam[i])))
            r = vr[:, j] / np.vdot(L[:, i], vr[:, j])           # L_i^H R_i(t) = 1
            q = vl[:, j] / np.conj(np.vdot(vl[:, j], R[:, i]))  # L_i(t)^H R_i = 1
            cols[s] = (r, q)
        fd_r = (cols[1.0][0] - cols[-1.0][0]) / (2 * h)
        fd_l = (np.vdot(cols[1.0][1], x) - np.vdot(cols[-1.0][1], x)) / (2 * h)
        assert np.linalg.norm(fd_r - dR[:, i]) < 1e-5 * np.linalg.norm(dR[:, i]), i
        dLx_want[i] = fd_l
    assert np.abs(dLx(x) - dLx_want).max() < 1e-5 * np.abs(dLx_want).max()


def test_full_deflation_is_the_exact_block_sign():
    """l = n: the exact part alone is sgn(B)(x1, x2) = (sgn(H) x1 + L_sgn(H, dH) x2, sgn(H) x2)
    (Theorem 1, the Frechet derivative by the block-matrix sign)."""
    dims, mass, mu, U, dU, op, x1, psi = _defl_problem()
    n = psi.size
    res = BD.deflated_block_sign(op, U, dU, x1, psi, 4, n, dims, mass, mu)
    H, dH = res["H"], res["dH"]
    S = SG.sign_schur(H)
    want1 = S @ x1.ravel() + SG.frechet_sign(H, dH) @ psi.ravel()
    want2 = S @ psi.ravel()
    assert np.linalg.norm(res["y1"].ravel() - want1) < 1e-10 * np.linalg.norm(want1)
    assert np.linalg.norm(res["y2"].ravel() - want2) < 1e-10 * np.linalg.norm(want2)


def test_projected_source_has_no_deflated_component():
    """Pbar x carries no component along the deflated invariant subspace of B: both
    coefficients c1, c2 of the projected source vanish (they would not if each pair's
    part were subtracted from x1 before the next c1 is formed)."""
    dims, mass, mu, U, dU, op, x1, psi = _defl_problem()
    l = 10
    res = BD.deflated_block_sign(op, U, dU, x1, psi, 8, l, dims, mass, mu)
    lam, R, L, dR, dLx = BD.eigenvector_derivatives(res["H"], res["dH"], l)
    p1, p2 = res["p1"], res["p2"]
    c2p = L.conj().T @ p2
    c1p = L.conj().T @ p1 + dLx(p2)
    scale = np.abs(res["c1"]).max() + np.abs(res["c2"]).max()
    assert np.abs(c2p).max() < 1e-12 * scale and np.abs(c1p).max() < 1e-10 * scale
    # the listing's sequential subtraction leaves the cross terms in c1
    x1s = x1.ravel().astype(np.complex128)
    c1_seq = np.zeros(l, dtype=np.complex128)
    c2 = res["c2"]
    dlx2 = dLx(psi.ravel())
    for i in range(l):
        c1_seq[i] = np.vdot(L[:, i], x1s) + dlx2[i]
        x1s = x1s - c1_seq[i] * R[:, i] - c2[i] * dR[:, i]
    assert np.abs(c1_seq - res["c1"]).max() > 1e-6 * scale


def test_deflation_improves_the_block_sign_at_fixed_k():
    dims, mass, mu, U, dU, op, x1, psi = _defl_problem()
    H = W.dense_h(U, dims, mass, mu)
    dH = W.dense_h(U + dU, dims, mass, mu) - H
    S = SG.sign_schur(H)
    want = np.concatenate([S @ x1.ravel() + SG.frechet_sign(H, dH) @ psi.ravel(), S @ psi.ravel()])
    errs = []
    for l in (0, 10, 40):
        res = BD.deflated_block_sign(op, U, dU, x1, psi, 24, l, dims, mass, mu)
        got = np.concatenate([res["y1"].ravel(), res["y2"].ravel()])
        errs.append(np.linalg.norm(got - want) / np.linalg.norm(want))
    assert errs[2] < errs[1] < errs[0], errs
    # eps_B of the deflated process (App. E's reason for general sources): falls with l
    e0 = BD.eps_block_deflated(op, U, dU, psi, 24, 0, dims, mass, mu)
    e40 = BD.eps_block_deflated(op, U, dU, psi, 24, 40, dims, mass, mu)
    assert e40 < e0
    assert BD.eps_block_deflated(op, U, dU, psi, 4, psi.size, dims, mass, mu) < 1e-12
