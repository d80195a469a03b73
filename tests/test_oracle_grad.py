"""Pins of the oracle derivative of S_k = Re <eta|TSL_k(H(U), psi)> over all links.

* torch's complex-gradient convention matches G = dS/dRe U + i dS/dIm U;
* the Theorem-1 backward of sgn(T) against finite differences;
* autograd G against central finite differences along su(3) and U(1) link
  directions (two step sizes, to show S_k is smooth there);
* the U(1) Ward identity at every site (gauge invariance, Sec. 4.3);
* the exact (Daleckii-Krein) gradient of Re eta^H sgn(H) psi against finite
  differences of the dense exact sign, and the TSL gradient with the full
  Krylov space against it.
"""
import numpy as np
import pytest
import torch

from oracle import grad as GR
from oracle import sign as SG
from oracle import tsl as T
from oracle import wilson as W
from synthetic import random_links, z2_complex_source


def test_torch_complex_gradient_convention():
    z = torch.tensor(1.0 + 2.0j, dtype=torch.complex128, requires_grad=True)
    (z.abs() ** 2).backward()
    assert complex(z.grad) == pytest.approx(2.0 + 4.0j)
    z2 = torch.tensor(0.3 - 0.7j, dtype=torch.complex128, requires_grad=True)
    torch.real(z2 * (2 - 1j)).backward()   # Re(c z): dS/dRe = Re c, dS/dIm = -Im c
    assert complex(z2.grad) == pytest.approx(2.0 + 1.0j)


def test_sign_matrix_backward(rng):
    n = 10
    w = rng.uniform(0.3, 2, n) * rng.choice([-1, 1], n) + 1j * rng.uniform(-1, 1, n)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = X @ np.diag(w) @ np.linalg.inv(X)
    C = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Tt = torch.from_numpy(A).requires_grad_(True)
    L = torch.real(torch.sum(torch.from_numpy(C) * T.sign_matrix(Tt)))
    L.backward()
    f = lambda M: np.real(np.sum(C * SG.sign_schur(M)))  # noqa: E731
    h = 1e-6
    fd = (f(A + h * E) - f(A - h * E)) / (2 * h)
    ad = np.real(np.sum(Tt.grad.numpy().conj() * E))
    assert abs(fd - ad) < 1e-7 * max(1.0, abs(ad))


@pytest.fixture(scope="module")
def small_case():
    dims = (3, 2, 2, 4)
    V = int(np.prod(dims))
    r = np.random.default_rng(77)
    U = random_links(dims, 0.5, r)
    psi = z2_complex_source(V, r)
    eta = z2_complex_source(V, r)
    op = W.WilsonOperator(dims, -2.0, 0.3)
    k = 20
    out = GR.grad_autograd(op, U, psi, eta, k)
    return dict(dims=dims, U=U, psi=psi, eta=eta, op=op, k=k, **out)


def test_autograd_against_finite_differences(small_case):
    c = small_case
    op, U, k = c["op"], c["U"], c["k"]
    S_of_U = lambda Uc: GR.objective(op, torch.from_numpy(Uc), torch.from_numpy(c["psi"]),  # noqa: E731
                                     torch.from_numpy(c["eta"]), k)[0].item()
    r = np.random.default_rng(8)
    ad, fd4, fd5 = [], [], []
    for _ in range(6):
        nu, site = int(r.integers(0, 4)), int(r.integers(0, op.volume))
        for X in (GR.su3_direction(r), np.eye(3, dtype=complex)):
            ad.append(GR.directional_from_gradient(c["G"], U, nu, site, X))
            fd5.append(GR.fd_directional(S_of_U, U, nu, site, X, 1e-5))
            fd4.append(GR.fd_directional(S_of_U, U, nu, site, X, 1e-4))
    ad, fd4, fd5 = map(np.array, (ad, fd4, fd5))
    assert np.linalg.norm(fd4 - fd5) / np.linalg.norm(fd5) < 1e-6   # smooth in h
    assert np.linalg.norm(ad - fd5) / np.linalg.norm(fd5) < 1e-6


def test_ward_identity_every_site(small_case):
    c = small_case
    lhs, rhs = GR.ward_residual(c["op"], c["G"], c["U"], c["psi"], c["eta"], c["y"], c["dpsi"])
    assert np.abs(lhs).max() > 1e-2          # non-trivial currents
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


def test_ward_identity_catches_a_planted_error(small_case):
    c = small_case
    G = c["G"].copy()
    G[1, 5] *= 1.001                          # perturb one link's gradient
    lhs, rhs = GR.ward_residual(c["op"], G, c["U"], c["psi"], c["eta"], c["y"], c["dpsi"])
    assert np.abs(lhs - rhs).max() > 1e-6


@pytest.fixture(scope="module")
def tiny_exact():
    dims = (2, 2, 2, 4)
    V = 32
    r = np.random.default_rng(5)
    U = random_links(dims, 0.5, r)
    psi = z2_complex_source(V, r)
    eta = z2_complex_source(V, r)
    G = GR.exact_gradient(U, psi, eta, dims, -2.0, 0.3)
    return dims, U, psi, eta, G


def test_exact_gradient_against_finite_differences(tiny_exact):
    dims, U, psi, eta, G = tiny_exact
    S = lambda Uc: GR.exact_objective(Uc, psi, eta, dims, -2.0, 0.3)  # noqa: E731
    r = np.random.default_rng(9)
    for _ in range(2):
        nu, site = int(r.integers(0, 4)), int(r.integers(0, 32))
        X = GR.su3_direction(r)
        fd = GR.fd_directional(S, U, nu, site, X, 1e-5)
        assert abs(GR.directional_from_gradient(G, U, nu, site, X) - fd) < 1e-6 * max(1, abs(fd))


def test_full_krylov_gradient_equals_exact(tiny_exact):
    dims, U, psi, eta, G = tiny_exact
    op = W.WilsonOperator(dims, -2.0, 0.3)
    out = GR.grad_autograd(op, U, psi, eta, 12 * 32, reorth=True)
    assert out["k_used"] >= 12 * 32 - 1
    assert np.linalg.norm(out["G"] - G) / np.linalg.norm(G) < 1e-6
