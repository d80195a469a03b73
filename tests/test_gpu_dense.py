"""GPU projected-matrix step: sgn(T) by scaled Newton and L_sgn(T, E) by Theorem 1,
against the oracle's Schur method and block-Schur Frechet derivative.

Sizes span one panel (k = 1, 7), several panels with a ragged last panel
(k = 37, 130), the workload sizes 64 and 200, the 512-thread register panel
(k = 300, 450) and the LDS panel beyond it (k = 600); a Lanczos matrix from the
4^4 workload is included, and matrices with zero diagonal blocks, whose every
elimination step needs a row exchange (a wrong pivot choice meets a zero pivot).
Tolerance: 1e-11 relative (Frobenius) for these well-separated spectra (Newton
and Schur differ by rounding times the condition number of the sign).
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import grad as GR
from oracle import sign as SG
from oracle.wilson import WilsonOperator
from synthetic import workload

pytestmark = pytest.mark.gpu


def _matrix(k, rng):
    w = rng.uniform(0.2, 2.0, k) * rng.choice([-1, 1], k) + 1j * rng.uniform(-1.5, 1.5, k)
    X = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)) + 2 * np.sqrt(k) * np.eye(k)
    return X @ np.diag(w) @ np.linalg.inv(X)


@pytest.fixture(scope="module")
def ctx():
    from paper_1604_08057_amd import Context
    c = Context((2, 2, 2, 2), -2.0, 0.0)
    yield c
    c.close()


@pytest.mark.parametrize("k", [1, 7, 37, 64, 130, 200, 300, 450, 600])
def test_dense_sign_and_frechet(ctx, k):
    say(f"dense sign k={k}")
    rng = np.random.default_rng(k)
    A = _matrix(k, rng)
    E = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    S, L, iters = ctx.dense_sign(dev(A), dev(E))
    S, L = host(S), host(L)
    S_ref = SG.sign_schur(A)
    L_ref = SG.frechet_sign(A, E)
    if k == 1:   # sgn is locally constant: the derivative of a scalar sign vanishes
        assert np.abs(L).max() < 1e-14 and np.abs(S - S_ref).max() < 1e-14
        return
    say(f"  iters={iters} sign err {rel(S, S_ref):.2e} frechet err {rel(L, L_ref):.2e}")
    assert rel(S, S_ref) < 1e-11
    assert rel(L, L_ref) < 1e-10


@pytest.mark.parametrize("k", [200, 300])
def test_dense_sign_needs_pivoting(ctx, k):
    # A = [[0, B], [C, 0]]: A^2 = diag(BC, CB), so sgn(A) = A (A^2)^{-1/2} is defined
    # when BC has no eigenvalue on the negative real axis; B, C near the identity
    h = k // 2
    rng = np.random.default_rng(k + 1)
    B = np.eye(h) + 0.3 * (rng.standard_normal((h, h)) + 1j * rng.standard_normal((h, h))) / np.sqrt(h)
    C = np.eye(h) + 0.3 * (rng.standard_normal((h, h)) + 1j * rng.standard_normal((h, h))) / np.sqrt(h)
    A = np.zeros((k, k), dtype=complex)
    A[:h, h:] = B
    A[h:, :h] = C
    say(f"dense sign with zero diagonal blocks k={k}")
    S, _, iters = ctx.dense_sign(dev(A))
    e = rel(host(S), SG.sign_schur(A))
    say(f"  iters={iters} sign err {e:.2e}")
    assert e < 1e-11


def test_dense_sign_of_lanczos_matrix(ctx):
    wl = workload(1)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    T = GR.forward(op, wl.links(), wl.psi(), wl.k)["T"]
    S, _, _ = ctx.dense_sign(dev(T))
    assert rel(host(S), SG.sign_schur(T)) < 1e-12


def test_dense_sign_rejects_bad_k(ctx):
    from paper_1604_08057_amd.tslov import TslovError
    with pytest.raises(TslovError):
        ctx.dense_sign(torch.zeros((1025, 1025), dtype=torch.complex128, device="cuda"))
