"""Pins of the oracle matrix sign function and Theorem 1 (Sec. 2).

Three independent evaluations (Schur, eigen-decomposition, Newton) agree;
sgn^2 = 1; a defective (Jordan) matrix; the Frechet derivative from Theorem 1
against Daleckii-Krein and finite differences; and, on tiny lattices, the
overlap identities: Ginsparg-Wilson, the mu = 0 unit circle, sgn(H(-mu)) =
sgn(H(mu))^dagger and the free-field closed form sgn(g5 D(p)) = g5 D(p)/sqrt(c).
"""
import math

import numpy as np
import pytest

from oracle import sign as SG
from oracle import wilson as W
from synthetic import random_links


def _random_nonnormal(n, rng, gap=0.3):
    w = rng.uniform(gap, 2.0, n) * rng.choice([-1, 1], n) + 1j * rng.uniform(-2, 2, n)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    X += 3 * np.eye(n)
    return X @ np.diag(w) @ np.linalg.inv(X)


def test_three_methods_agree(rng):
    A = _random_nonnormal(60, rng)
    S1 = SG.sign_schur(A)
    S2 = SG.sign_eig(A)
    S3 = SG.sign_newton(A)
    scale = np.linalg.norm(S1)
    assert np.linalg.norm(S1 - S2) / scale < 1e-11
    assert np.linalg.norm(S1 - S3) / scale < 1e-11
    assert np.linalg.norm(S1 @ S1 - np.eye(60)) < 1e-10


def test_diagonal_and_jordan_block():
    d = np.diag([1.5 + 2j, -0.1 + 0j, 0.2 - 5j, -3 - 1j])
    assert np.allclose(SG.sign_schur(d), np.diag([1, -1, 1, -1]))
    J = np.array([[0.7, 1.0, 0.0], [0.0, 0.7, 1.0], [0.0, 0.0, 0.7]], dtype=complex)
    assert np.allclose(SG.sign_schur(J), np.eye(3), atol=1e-14)
    # two Jordan blocks of opposite sign: sgn commutes with A and squares to 1
    A = np.zeros((4, 4), complex)
    A[:2, :2] = [[0.5, 1.0], [0.0, 0.5]]
    A[2:, 2:] = [[-0.4, 1.0], [0.0, -0.4]]
    A[0, 3] = 0.8
    S = SG.sign_schur(A)
    assert np.allclose(S @ S, np.eye(4), atol=1e-13)
    assert np.allclose(S @ A, A @ S, atol=1e-13)
    assert np.allclose(np.trace(S), 0)


def test_sign_undefined_on_axis():
    with pytest.raises(SG.SignUndefined):
        SG.sign_schur(np.diag([1.0, 1e-20 + 1j, -2.0]).astype(complex))


def test_theorem1_frechet(rng):
    n = 24
    A = _random_nonnormal(n, rng)
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    L1 = SG.frechet_sign(A, E)
    L2 = SG.daleckii_krein(A, E)
    h = 1e-6
    L3 = (SG.sign_schur(A + h * E) - SG.sign_schur(A - h * E)) / (2 * h)
    s = np.linalg.norm(L1)
    assert np.linalg.norm(L1 - L2) / s < 1e-10
    assert np.linalg.norm(L1 - L3) / s < 1e-7
    # trace identity tr(L(A,E) B) = tr(E L(A,B)) used by the adjoint
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    assert abs(np.trace(L1 @ B) - np.trace(E @ SG.frechet_sign(A, B))) < 1e-9 * s * np.linalg.norm(B)


@pytest.fixture(scope="module")
def tiny_overlap():
    dims = (2, 2, 2, 4)
    U = random_links(dims, 0.5, np.random.default_rng(11))
    out = {}
    for mu in (0.0, 0.3, -0.3):
        H = W.dense_h(U, dims, -2.0, mu)
        out[mu] = (H, SG.sign_schur(H))
    return dims, U, out


def test_overlap_identities(tiny_overlap):
    dims, U, out = tiny_overlap
    V = int(np.prod(dims))
    n = 12 * V
    g5 = np.kron(np.eye(V), np.kron(W.gamma5(), np.eye(3)))
    for mu in (0.0, 0.3):
        H, S = out[mu]
        assert np.abs(S @ S - np.eye(n)).max() < 1e-11
        D = np.eye(n) + g5 @ S  # overlap operator, a = 1 (eq. overlap)
        gw = g5 @ D + D @ g5 - D @ g5 @ D
        assert np.abs(gw).max() < 1e-11
    # mu = 0: H Hermitian, S Hermitian, spectrum of D_ov on the circle |z - 1| = 1
    H0, S0 = out[0.0]
    assert np.abs(S0 - S0.conj().T).max() < 1e-11
    ev = np.linalg.eigvals(np.eye(n) + g5 @ S0)
    assert np.abs(np.abs(ev - 1) - 1).max() < 1e-10
    # sgn(H(-mu)) = sgn(H(mu))^dagger since H(-mu) = H(mu)^dagger
    assert np.abs(out[-0.3][1] - out[0.3][1].conj().T).max() < 1e-11
    # Schur vs eigen-decomposition on the Wilson operator itself
    assert np.abs(SG.sign_eig(out[0.3][0]) - out[0.3][1]).max() < 1e-10


def test_free_field_sign_closed_form():
    dims = (2, 2, 2, 4)
    V = int(np.prod(dims))
    mu = 0.3
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    S = SG.sign_schur(W.dense_h(U, dims, -1.5, mu))
    g5 = W.gamma5()
    rng = np.random.default_rng(3)
    for _ in range(3):
        n = [rng.integers(0, d) for d in dims]
        p = [2 * math.pi * n[i] / dims[i] for i in range(3)] + [math.pi * (2 * n[3] + 1) / dims[3]]
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        h = g5 @ W.free_field_symbol(p, -1.5, mu)
        pt = np.array(p, dtype=complex)
        pt[3] -= 1j * mu
        kap = W.kappa_of_mass(-1.5)
        a = 1 - 2 * kap * np.sum(np.cos(pt))
        c = a ** 2 + np.sum((2 * kap * np.sin(pt)) ** 2)
        assert np.allclose(h @ h, c * np.eye(4))   # (g5 D(p))^2 is a scalar
        root = np.sqrt(c)                           # principal root: sgn(Re) of eigenvalues +-sqrt(c)
        want = W.plane_wave(dims, p, (h / root) @ chi)
        got = (S @ W.plane_wave(dims, p, chi).ravel()).reshape(V, 4, 3)
        assert np.abs(got - want).max() < 1e-11
