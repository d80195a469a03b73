"""Pins of oracle.constfield: exact eigenpairs and sign of H on a gauge-rotated constant field.

* the closed-form spectrum (one 12 x 12 matrix per momentum) equals the
  eigenvalues of the oracle's dense H, built link by link, on a ragged lattice;
* the closed-form right and left eigenvectors satisfy H R = lambda R and
  H^dag L = conj(lambda) L under the oracle's gather stencil and L^H R = I, on a
  ragged lattice (odd and even extents, antiperiodic time);
* the spectral sign equals the Schur sign of the dense H, and squares to 1;
* commuting constant links (an abelian background) give doubly degenerate
  eigenvalues, non-commuting ones do not;
* eigenpairs tracked to a moved constant field are eigenpairs of the moved dense H.
The field itself comes from synthetic.rotated_constant_links (not from the oracle).
"""
import numpy as np
import pytest
import torch
from scipy.linalg import expm
from scipy.optimize import linear_sum_assignment

from oracle import constfield as CF
from oracle.sign import sign_schur
from oracle.wilson import WilsonOperator, dense_h
from synthetic.fields import links_from_constant, random_su3, rotated_constant_links

MASS, MU = -2.0, 0.3


@pytest.fixture(scope="module")
def field():
    dims = (3, 2, 4, 4)
    U, C, g = rotated_constant_links(dims, 0.8, np.random.default_rng(5))
    return dims, U, C, g, dense_h(U, dims, MASS, MU)


def test_spectrum_matches_dense_eigenvalues(field):
    dims, U, C, g, H = field
    ev = np.linalg.eigvals(H)
    lam, _, _ = CF.spectrum(dims, MASS, MU, C)
    cost = np.abs(ev[:, None] - lam.ravel()[None, :])
    r, c = linear_sum_assignment(cost)
    assert cost[r, c].max() < 1e-12


def test_eigenvectors_under_gather_stencil():
    dims = (3, 2, 5, 6)
    U, C, g = rotated_constant_links(dims, 0.8, np.random.default_rng(9))
    res = CF.lowest_eigenpairs(dims, MASS, MU, C, g, 12)
    op = WilsonOperator(dims, MASS, MU)
    Ut = torch.from_numpy(U)
    for i in range(12):
        r, q = torch.from_numpy(res["R"][i]), torch.from_numpy(res["L"][i])
        assert (op.h(Ut, r) - res["lam"][i] * r).norm().item() < 1e-12 * r.norm().item()
        assert (op.h_dag(Ut, q) - np.conj(res["lam"][i]) * q).norm().item() < 1e-12 * q.norm().item()
    G = res["L"].reshape(12, -1).conj() @ res["R"].reshape(12, -1).T
    assert np.abs(G - np.eye(12)).max() < 1e-12
    assert np.all(np.diff(np.abs(res["lam"])) >= 0) and res["edge"][0] <= res["edge"][1]


def test_spectral_sign_matches_schur(field):
    dims, U, C, g, H = field
    V = int(np.prod(dims))
    psi = np.random.default_rng(1).standard_normal((V, 4, 3)) + 1j * np.random.default_rng(2).standard_normal((V, 4, 3))
    y = CF.exact_sign(dims, MASS, MU, C, g, psi)
    want = (sign_schur(H) @ psi.ravel()).reshape(psi.shape)
    assert np.linalg.norm(y - want) < 1e-12 * np.linalg.norm(want)
    z = CF.exact_sign(dims, MASS, MU, C, g, y)
    assert np.linalg.norm(z - psi) < 1e-12 * np.linalg.norm(psi)


def test_abelian_background_is_degenerate_in_spin():
    dims = (2, 2, 2, 4)
    r = np.random.default_rng(4)
    ph = r.uniform(-1, 1, (4, 2))
    C = np.stack([np.diag(np.exp(1j * np.array([a, b, -a - b]))) for a, b in ph])
    lam, _, _ = CF.spectrum(dims, MASS, MU, C)
    for q in range(lam.shape[0]):
        s = np.sort_complex(lam[q])
        assert np.abs(s[0::2] - s[1::2]).max() < 1e-10
    lam2, _, _ = CF.spectrum(dims, MASS, MU, random_su3(4, 0.8, r))
    s = np.sort_complex(lam2.ravel())
    assert np.abs(np.diff(s)).min() > 1e-8


def test_tracked_eigenpairs_of_moved_field(field):
    dims, U, C, g, H = field
    res = CF.lowest_eigenpairs(dims, MASS, MU, C, g, 6)
    X = np.array([[0.3, 0.1 - 0.2j, 0], [0.1 + 0.2j, -0.5, 0.4j], [0, -0.4j, 0.2]])
    for nu in (0, 3):
        Ct = C.copy()
        Ct[nu] = expm(1j * 1e-3 * X) @ C[nu]
        lam, R, L, jump = CF.tracked_eigenpairs(dims, MASS, MU, Ct, g, res["labels"], res["lam"])
        Ht = dense_h(links_from_constant(Ct, g, dims), dims, MASS, MU)
        assert 0 < jump < 1e-2
        for i in range(6):
            assert np.linalg.norm(Ht @ R[i].ravel() - lam[i] * R[i].ravel()) < 1e-13
            assert np.linalg.norm(Ht.conj().T @ L[i].ravel() - np.conj(lam[i]) * L[i].ravel()) < 1e-12 * np.linalg.norm(L[i])
