"""Pins of the oracle two-sided Lanczos approximation (Sec. 2, Sec. 4.1).

The TSL result is basis-free: it equals the oblique (Petrov-Galerkin)
projection onto K_k(A, x) along K_k(A^H, x), built here from QR-orthonormalised
power bases, and equals p(A) x with p interpolating sgn at the Ritz values.
Special cases: an eigenvector source (lucky breakdown at j = 1), a free-field
plane wave (exact at k = 2), the full space with re-biorthogonalisation (equals
the exact sign), gauge covariance and invariance under positive scaling.
"""
import math

import numpy as np
import pytest
import torch

from oracle import sign as SG
from oracle import tsl as T
from oracle import wilson as W
from synthetic import random_links, random_su3, workload


def _dense_problem(n, rng):
    w = rng.uniform(0.2, 2.0, n) * rng.choice([-1, 1], n) + 1j * rng.uniform(-1, 1, n)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    A = X @ np.diag(w) @ np.linalg.inv(X)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, x, w, X


def test_ritz_interpolation_and_oblique_projection(rng):
    A, x, _, _ = _dense_problem(60, rng)
    k = 12
    res = T.tsl_dense(A, x, k)
    y = res.y.numpy()
    ritz = np.linalg.eigvals(res.T.numpy())
    y_interp = T.ritz_interpolation(A, x, ritz)
    assert np.linalg.norm(y - y_interp) / np.linalg.norm(y) < 1e-10
    # oblique projection from orthonormal power bases, no Lanczos vectors involved
    K = np.stack([np.linalg.matrix_power(A, i) @ x for i in range(k)], 1)
    L = np.stack([np.linalg.matrix_power(A.conj().T, i) @ x for i in range(k)], 1)
    Q, _ = np.linalg.qr(K)
    P, _ = np.linalg.qr(L)
    G = np.linalg.inv(P.conj().T @ Q)
    M = G @ P.conj().T @ A @ Q
    z = G @ P.conj().T @ x
    y_proj = Q @ SG.sign_schur(M) @ z
    assert np.linalg.norm(y - y_proj) / np.linalg.norm(y) < 1e-9
    # biorthogonality of the computed bases
    Vm = torch.stack(res.V, 1).numpy()
    Wm = torch.stack(res.W, 1).numpy()
    assert np.abs(Wm.conj().T @ Vm - np.eye(k)).max() < 1e-10
    assert np.abs(Wm.conj().T @ A @ Vm - res.T.numpy()).max() < 1e-9


def test_eigenvector_source_lucky_breakdown(rng):
    A, _, w, X = _dense_problem(30, rng)
    i = 3
    res = T.tsl_dense(A, X[:, i], 10)
    assert res.k_used == 1 and res.breakdown == 1
    assert np.allclose(res.y.numpy(), np.sign(w[i].real) * X[:, i], atol=1e-12)


def test_free_field_plane_wave_exact_at_k2():
    dims = (4, 4, 4, 4)
    V = 256
    mu, mass = 0.3, -1.5
    U = torch.from_numpy(np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy())
    op = W.WilsonOperator(dims, mass, mu)
    p = [2 * math.pi / 4, 0.0, 2 * math.pi * 2 / 4, math.pi * 3 / 4]
    chi = np.arange(12).reshape(4, 3) * (0.3 + 0.1j) + 1.0
    psi = torch.from_numpy(W.plane_wave(dims, p, chi))
    res = T.tsl_wilson(op, U, psi, 20)
    assert res.k_used == 2 and res.breakdown == 1
    h = W.gamma5() @ W.free_field_symbol(p, mass, mu)
    want = W.plane_wave(dims, p, (h / np.sqrt((h @ h)[0, 0])) @ chi)
    assert np.abs(res.y.numpy() - want).max() < 1e-12


def test_full_space_with_reorthogonalisation_is_exact(rng):
    A, x, _, _ = _dense_problem(40, rng)
    res = T.tsl_dense(A, x, 40, reorth=True)
    exact = SG.sign_schur(A) @ x
    assert np.linalg.norm(res.y.numpy() - exact) / np.linalg.norm(exact) < 1e-9


def test_gauge_covariance_and_scale_invariance(rng):
    dims = (3, 2, 4, 4)
    V = int(np.prod(dims))
    U = random_links(dims, 0.5, rng)
    psi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    op = W.WilsonOperator(dims, -2.0, 0.3)
    g = random_su3(V, 1.0, rng)
    Ug = np.einsum("vab,nvbc,nvdc->nvad", g, U, g[op.geom.fwd].conj())
    gpsi = np.einsum("vab,vsb->vsa", g, psi)
    with torch.no_grad():
        y = T.tsl_wilson(op, torch.from_numpy(U), torch.from_numpy(psi), 24).y.numpy()
        yg = T.tsl_wilson(op, torch.from_numpy(Ug), torch.from_numpy(gpsi), 24).y.numpy()
    assert np.abs(yg - np.einsum("vab,vsb->vsa", g, y)).max() < 1e-10 * np.abs(y).max()
    A = W.dense_h(U, dims, -2.0, 0.3)
    r1 = T.tsl_dense(A, psi.ravel(), 24).y.numpy()
    r2 = T.tsl_dense(2.5 * A, psi.ravel(), 24).y.numpy()
    assert np.linalg.norm(r1 - y.ravel()) / np.linalg.norm(r1) < 1e-11
    assert np.linalg.norm(r1 - r2) / np.linalg.norm(r1) < 1e-10


def test_reduction_order_sensitivity_tiny_config():
    """The same TSL with a permuted dot-product order: sigma stays far below 1e-10."""
    wl = workload(1)
    op = W.WilsonOperator(wl.dims, wl.mass, wl.mu)
    U, psi = torch.from_numpy(wl.links()), torch.from_numpy(wl.psi())
    perm = np.random.default_rng(0).permutation(12 * wl.volume)
    with torch.no_grad():
        y0 = T.tsl_wilson(op, U, psi, wl.k).y.numpy()
        y1 = T.tsl_wilson(op, U, psi, wl.k, perm=perm).y.numpy()
    sigma = np.linalg.norm(y0 - y1) / np.linalg.norm(y0)
    assert sigma < 1e-11
