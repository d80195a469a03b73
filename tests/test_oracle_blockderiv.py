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
