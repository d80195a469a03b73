"""Pins of the oracle derivative of the deflated sign function (eigenpair motion included).

* l = n: every eigenpair is deflated, S is the exact Re eta^H sgn(H) psi and the
  gradient equals the Daleckii-Krein gradient of the exact sign (an independent
  formula: divided differences of sgn on the spectrum);
* l = 10, k = 24: central finite differences of S with the eigenpairs recomputed
  at U +- h X along random su(3) and U(1) link directions (h = 1e-5);
* the gradient does not depend on the eigenvector normalisation (R_i -> t R_i,
  L_i -> L_i / conj(t) leaves every Pi_i unchanged);
* the source gradient against finite differences of S in psi.
"""
import numpy as np
import pytest

from oracle import deflation as DF
from oracle import grad as GR
from synthetic import random_links, z2_complex_source

DIMS, MASS, MU = (2, 2, 2, 4), -2.0, 0.3


@pytest.fixture(scope="module")
def case():
    r = np.random.default_rng(31)
    U = random_links(DIMS, 0.5, r)
    psi = z2_complex_source(32, r)
    eta = z2_complex_source(32, r)
    return U, psi, eta


def test_full_deflation_gradient_is_exact(case):
    U, psi, eta = case
    G, S, _ = DF.deflated_gradient(U, psi, eta, 8, DIMS, MASS, MU, 384)
    assert abs(S - GR.exact_objective(U, psi, eta, DIMS, MASS, MU)) < 1e-9 * abs(S)
    Gx = GR.exact_gradient(U, psi, eta, DIMS, MASS, MU)
    assert np.linalg.norm(G - Gx) / np.linalg.norm(Gx) < 1e-8


def test_finite_differences(case):
    U, psi, eta = case
    l, k = 10, 24
    G, S, _ = DF.deflated_gradient(U, psi, eta, k, DIMS, MASS, MU, l)
    f = lambda Uh: DF.deflated_objective(Uh, psi, eta, k, DIMS, MASS, MU, l)
    assert abs(f(U) - S) < 1e-10 * abs(S)
    r = np.random.default_rng(5)
    errs = []
    for t in range(6):
        nu, site = int(r.integers(4)), int(r.integers(32))
        X = GR.su3_direction(r) if t % 2 == 0 else np.eye(3)
        fd = GR.fd_directional(f, U, nu, site, X, h=1e-5)
        an = GR.directional_from_gradient(G, U, nu, site, X)
        errs.append(abs(fd - an) / max(abs(an), 1e-3 * np.abs(G).max()))
    assert max(errs) < 1e-5, errs


def test_normalisation_independence(case):
    U, psi, eta = case
    from oracle.wilson import dense_h
    G1, S1, _ = DF.deflated_gradient(U, psi, eta, 16, DIMS, MASS, MU, 6)
    # deflated_gradient normalises internally; check the projector form directly
    H = dense_h(U, DIMS, MASS, MU)
    lam, R, L = DF.eigenpairs(H, 6)
    t = np.exp(0.7j) * np.linspace(0.5, 2.0, 6)
    assert np.allclose((R * t) @ (L / t.conj()).conj().T, R @ L.conj().T, atol=1e-12)
    Zs, _ = DF.reduced_resolvents(H, range(6))
    for i in range(6):
        P = np.outer(R[:, i], L[:, i].conj())
        assert np.abs(P @ Zs[i]).max() < 1e-9 and np.abs(Zs[i] @ P).max() < 1e-9
        # (lambda - H) Z = 1 - Pi on the whole space
        assert np.abs((lam[i] * np.eye(384) - H) @ Zs[i] - (np.eye(384) - P)).max() < 1e-8


def test_source_gradient(case):
    U, psi, eta = case
    l, k = 10, 24
    _, S, pb = DF.deflated_gradient(U, psi, eta, k, DIMS, MASS, MU, l)
    r = np.random.default_rng(9)
    d = z2_complex_source(32, r)
    h = 1e-6
    f = lambda p: DF.deflated_objective(U, p, eta, k, DIMS, MASS, MU, l)
    fd = (f(psi + h * d) - f(psi - h * d)) / (2 * h)
    an = float(np.real(np.vdot(pb.ravel(), d.ravel())))
    assert abs(fd - an) < 1e-6 * abs(an)
