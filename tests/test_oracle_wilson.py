"""Pins of the oracle Wilson-Dirac operator (App. A, eq. WD_op/WD_G).

Each pin is something other than the oracle's own formula: the Clifford
algebra, an independent dense builder, g5-hermiticity, the free-field closed
form for plane waves (antiperiodic time momenta, p4 -> p4 - i mu) and gauge
covariance.  The last tests plant mistakes in copies of the oracle to show
that these pins catch them.
"""
import math

import numpy as np
import pytest
import torch

from oracle import wilson as W
from synthetic import random_links, random_su3, z2_complex_source

TINY = [(2, 2, 2, 4), (3, 2, 2, 4)]


def test_clifford_algebra_and_gamma5():
    g = W.gamma_matrices()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * (m == n) * np.eye(4), atol=1e-15)
    g5 = W.gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for m in range(4):
        assert np.allclose(g5 @ g[m] + g[m] @ g5, 0)


def test_kappa():
    assert W.kappa_of_mass(-2.0) == 0.25
    assert math.isclose(W.kappa_of_mass(0.0), 1 / 8)


@pytest.mark.parametrize("dims", TINY)
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_gather_matches_dense(dims, mu, rng):
    U = random_links(dims, 0.7, rng)
    V = int(np.prod(dims))
    psi = z2_complex_source(V, rng) + 0.3 * rng.standard_normal((V, 4, 3))
    op = W.WilsonOperator(dims, -2.0, mu)
    Dd = W.dense_dw(U, dims, -2.0, mu)
    got = op.dw(torch.from_numpy(U), torch.from_numpy(psi)).numpy().ravel()
    assert np.allclose(got, Dd @ psi.ravel(), atol=1e-14, rtol=0)
    Hd = W.dense_h(U, dims, -2.0, mu)
    got_h = op.h(torch.from_numpy(U), torch.from_numpy(psi)).numpy().ravel()
    assert np.allclose(got_h, Hd @ psi.ravel(), atol=1e-14, rtol=0)
    got_hd = op.h_dag(torch.from_numpy(U), torch.from_numpy(psi)).numpy().ravel()
    assert np.allclose(got_hd, Hd.conj().T @ psi.ravel(), atol=1e-14, rtol=0)


@pytest.mark.parametrize("mu", [0.0, 0.25])
def test_gamma5_hermiticity(mu, rng):
    dims = (2, 2, 2, 4)
    U = random_links(dims, 0.9, rng)
    V = 32
    g5 = np.kron(np.eye(V), np.kron(W.gamma5(), np.eye(3)))
    Dp = W.dense_dw(U, dims, -2.0, mu)
    Dm = W.dense_dw(U, dims, -2.0, -mu)
    assert np.abs(Dp.conj().T - g5 @ Dm @ g5).max() < 1e-15
    Hp = W.dense_h(U, dims, -2.0, mu)
    Hm = W.dense_h(U, dims, -2.0, -mu)
    assert np.abs(Hp.conj().T - Hm).max() < 1e-15
    if mu == 0.0:
        assert np.abs(Hp - Hp.conj().T).max() < 1e-15


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 2, 6)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_plane_waves(dims, mu, rng):
    V = int(np.prod(dims))
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    op = W.WilsonOperator(dims, -2.0, mu)
    for _ in range(4):
        n = [rng.integers(0, d) for d in dims]
        p = [2 * math.pi * n[i] / dims[i] for i in range(3)] + [math.pi * (2 * n[3] + 1) / dims[3]]
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = W.plane_wave(dims, p, chi)
        got = op.dw(torch.from_numpy(U), torch.from_numpy(psi)).numpy()
        want = W.plane_wave(dims, p, W.free_field_symbol(p, -2.0, mu) @ chi)
        assert np.abs(got - want).max() < 1e-13


def test_gauge_covariance(rng):
    dims = (3, 4, 2, 4)
    V = int(np.prod(dims))
    U = random_links(dims, 0.6, rng)
    g = random_su3(V, 1.0, rng)
    op = W.WilsonOperator(dims, -2.0, 0.4)
    Ug = np.einsum("vab,nvbc,nvdc->nvad", g, U, g[op.geom.fwd].conj())
    psi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    gpsi = np.einsum("vab,vsb->vsa", g, psi)
    lhs = op.dw(torch.from_numpy(Ug), torch.from_numpy(gpsi)).numpy()
    rhs = np.einsum("vab,vsb->vsa", g, op.dw(torch.from_numpy(U), torch.from_numpy(psi)).numpy())
    assert np.abs(lhs - rhs).max() < 1e-13


# ---------------------------------------------------------------- planted mistakes

class _WrongProjector(W.WilsonOperator):
    """(1 - g) on the forward hop instead of (1 + g)."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.gam = -self.gam


class _WrongMuSign(W.WilsonOperator):
    def hop(self, U, psi, mu):
        return super().hop(U, psi, -mu)


class _WrongBackwardLink(W.WilsonOperator):
    """Uses U_nu(x)^dagger instead of U_nu(x - nu)^dagger on the backward hop."""

    def hop(self, U, psi, mu):
        out = torch.zeros_like(psi)
        for nu in range(4):
            ef = math.exp(mu) if nu == 3 else 1.0
            eb = math.exp(-mu) if nu == 3 else 1.0
            g = self.gam[nu]
            up = torch.einsum("vab,vsb->vsa", U[nu], psi[self.fwd[nu]])
            up = up + torch.einsum("st,vta->vsa", g, up)
            out = out + (ef * self.sf[nu])[:, None, None] * up
            dn = torch.einsum("vba,vsb->vsa", U[nu].conj(), psi[self.bwd[nu]])
            dn = dn - torch.einsum("st,vta->vsa", g, dn)
            out = out + (eb * self.sb[nu])[:, None, None] * dn
        return out


def _free_field_error(op_cls, dims=(4, 4, 4, 4), mu=0.3):
    V = int(np.prod(dims))
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    op = op_cls(dims, -2.0, mu)
    p = [2 * math.pi / 4, 0.0, 2 * math.pi * 3 / 4, math.pi * 3 / 4]
    chi = np.arange(12).reshape(4, 3) + 1j
    got = op.dw(torch.from_numpy(U), torch.from_numpy(W.plane_wave(dims, p, chi))).numpy()
    want = W.plane_wave(dims, p, W.free_field_symbol(p, -2.0, mu) @ chi)
    return np.abs(got - want).max()


def _covariance_error(op_cls):
    rng = np.random.default_rng(5)
    dims = (3, 4, 2, 4)
    V = int(np.prod(dims))
    U = random_links(dims, 0.6, rng)
    g = random_su3(V, 1.0, rng)
    op = op_cls(dims, -2.0, 0.4)
    Ug = np.einsum("vab,nvbc,nvdc->nvad", g, U, g[op.geom.fwd].conj())
    psi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    gpsi = np.einsum("vab,vsb->vsa", g, psi)
    lhs = op.dw(torch.from_numpy(Ug), torch.from_numpy(gpsi)).numpy()
    rhs = np.einsum("vab,vsb->vsa", g, op.dw(torch.from_numpy(U), torch.from_numpy(psi)).numpy())
    return np.abs(lhs - rhs).max()


def test_planted_mistakes_are_caught():
    assert _free_field_error(W.WilsonOperator) < 1e-13
    assert _free_field_error(_WrongProjector) > 1e-3
    assert _free_field_error(_WrongMuSign) > 1e-3
    assert _covariance_error(W.WilsonOperator) < 1e-13
    assert _covariance_error(_WrongBackwardLink) > 1e-3
