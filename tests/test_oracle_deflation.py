"""Pins of the oracle deflation and error estimate (Sec. 3, Sec. 4.1).

* eigenpairs: H R = R Lambda, L^H H = Lambda L^H, L^H R = 1;
* deflating every eigenpair reproduces the exact (Schur) sign;
* the projected source has no component along the deflated right eigenvectors;
* with the full complementary Krylov space (k = n - l, re-biorthogonalised) the
  deflated result is exact;
* deflating the smallest eigenvalues improves the approximation at fixed k;
* eps_A of the exact sign is zero, and eps_A tracks the true error.
"""
import numpy as np
import pytest
import torch

from oracle import deflation as DF
from oracle import sign as SG
from oracle import tsl as T
from oracle import wilson as W
from synthetic import random_links, z2_complex_source


@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 4)
    r = np.random.default_rng(21)
    U = random_links(dims, 0.5, r)
    psi = z2_complex_source(32, r)
    H = W.dense_h(U, dims, -2.0, 0.3)
    return dims, U, psi, H, SG.sign_schur(H)


def test_eigenpairs_are_biorthonormal(tiny):
    dims, U, psi, H, S = tiny
    lam, R, L = DF.eigenpairs(H, 12)
    assert np.allclose(L.conj().T @ R, np.eye(12), atol=1e-10)
    assert np.abs(H @ R - R * lam[None, :]).max() < 1e-10
    assert np.abs(L.conj().T @ H - lam[:, None] * L.conj().T).max() < 1e-10
    assert np.all(np.diff(np.abs(lam)) >= 0)


def test_full_deflation_is_exact(tiny):
    dims, U, psi, H, S = tiny
    n = H.shape[0]
    lam, R, L = DF.eigenpairs(H, n)
    op = W.WilsonOperator(dims, -2.0, 0.3)
    y = DF.deflated_sign(op, U, psi, 10, lam, R, L)
    exact = (S @ psi.ravel()).reshape(psi.shape)
    assert np.linalg.norm(y - exact) / np.linalg.norm(exact) < 1e-9


def test_projection_and_full_complement(tiny):
    dims, U, psi, H, S = tiny
    n, l = H.shape[0], 20
    lam, R, L = DF.eigenpairs(H, l)
    x = psi.ravel()
    xp = x - R @ (L.conj().T @ x)
    assert np.abs(L.conj().T @ xp).max() < 1e-12 * np.linalg.norm(x)
    op = W.WilsonOperator(dims, -2.0, 0.3)
    y = DF.deflated_sign(op, U, psi, n - l, lam, R, L, reorth=True)
    exact = (S @ x).reshape(psi.shape)
    assert np.linalg.norm(y - exact) / np.linalg.norm(exact) < 1e-7


def test_deflation_improves_accuracy(tiny):
    dims, U, psi, H, S = tiny
    op = W.WilsonOperator(dims, -2.0, 0.3)
    exact = (S @ psi.ravel()).reshape(psi.shape)
    k = 40
    with torch.no_grad():
        y0 = T.tsl_wilson(op, torch.from_numpy(U), torch.from_numpy(psi), k).y.numpy()
    lam, R, L = DF.eigenpairs(H, 40)
    y1 = DF.deflated_sign(op, U, psi, k, lam, R, L)
    e0 = np.linalg.norm(y0 - exact) / np.linalg.norm(exact)
    e1 = np.linalg.norm(y1 - exact) / np.linalg.norm(exact)
    assert e1 < 0.5 * e0


def test_error_estimate(tiny):
    dims, U, psi, H, S = tiny
    assert DF.error_estimate(lambda v: (S @ v.ravel()).reshape(v.shape), psi) < 1e-12
    # a gapped operator (m = -1, smooth links), where TSL converges with k
    r = np.random.default_rng(4)
    Ug = random_links(dims, 0.05, r)
    Hg = W.dense_h(Ug, dims, -1.0, 0.2)
    Sg = SG.sign_schur(Hg)
    op = W.WilsonOperator(dims, -1.0, 0.2)
    exact = (Sg @ psi.ravel()).reshape(psi.shape)

    def tsl_k(k):
        def f(v):
            with torch.no_grad():
                return T.tsl_wilson(op, torch.from_numpy(Ug), torch.from_numpy(v), k).y.numpy()
        return f

    errs, ests = [], []
    for k in (8, 16, 32, 64):
        errs.append(np.linalg.norm(tsl_k(k)(psi) - exact) / np.linalg.norm(exact))
        ests.append(DF.error_estimate(tsl_k(k), psi))
    assert all(np.diff(ests) < 0) and all(np.diff(errs) < 0)
    for e, a in zip(ests, errs):
        assert 0.3 * a < e < 3 * a   # the estimate tracks the true error
