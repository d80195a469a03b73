"""Pins of the oracle nested TSL (one level of nesting, Sec. 4.1 and the cited method).

* The transform it rests on: T (T^2)^{-1/2} = sgn(T) with the principal square
  root, against the Schur sign, on a Lanczos matrix of the 4^4 workload;
* the inner approximation is the oblique projection of W^{1/2} e_1 onto
  K_m(W, e_1) along K_m(W^H, e_1), built from QR-orthonormalised power bases
  (no Lanczos vectors), W = (T^2)^{-1};
* with k^I = k^O the nested result is the plain TSL result (the inner space is
  the whole space);
* as k^I grows the inner result converges to sgn(T) e_1 (monotone, below 1e-7
  at k^I = 100 on the 8^4 workload's T_200, k^O = 200);
* on the Wilson operator, nested y with a converged inner size equals plain y.
"""
import numpy as np
import scipy.linalg as sla

from oracle import grad as GR
from oracle import nested as N
from oracle.sign import sign_schur
from oracle.wilson import WilsonOperator
from synthetic import workload


def _T(config, k=None):
    wl = workload(config)
    return GR.forward(WilsonOperator(wl.dims, wl.mass, wl.mu), wl.links(), wl.psi(), k or wl.k)["T"]


def test_inverse_square_root_transform():
    T = _T(1)
    S = T @ sla.sqrtm(np.linalg.inv(T @ T))
    assert np.linalg.norm(S - sign_schur(T)) / np.linalg.norm(sign_schur(T)) < 1e-10


def test_inner_step_is_the_oblique_projection():
    T = _T(1, 40)
    k, m = T.shape[0], 6
    e1 = np.zeros(k, dtype=np.complex128)
    e1[0] = 1.0
    c, ku, _ = N.inner_sign_e1(T, m)
    W = np.linalg.inv(T @ T)
    K = np.stack([np.linalg.matrix_power(W, i) @ e1 for i in range(m)], 1)
    L = np.stack([np.linalg.matrix_power(W.conj().T, i) @ e1 for i in range(m)], 1)
    Q, _ = np.linalg.qr(K)
    P, _ = np.linalg.qr(L)
    G = np.linalg.inv(P.conj().T @ Q)
    M = G @ P.conj().T @ W @ Q
    z = G @ P.conj().T @ e1
    want = T @ (Q @ sla.sqrtm(M) @ z)
    assert ku == m
    assert np.linalg.norm(c - want) / np.linalg.norm(want) < 1e-8


def test_full_inner_space_is_plain_tsl():
    T = _T(1, 30)
    c, ku, _ = N.inner_sign_e1(T, 30)
    want = sign_schur(T)[:, 0]
    assert ku == 30
    assert np.linalg.norm(c - want) / np.linalg.norm(want) < 1e-9


def test_inner_size_converges():
    T = _T(2)                                       # 8^4 workload, k^O = 200
    want = sign_schur(T)[:, 0]
    errs = [np.linalg.norm(N.inner_sign_e1(T, m)[0] - want) / np.linalg.norm(want) for m in (25, 50, 100, 150)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[2] < 1e-7 and errs[3] < 1e-9, errs


def test_nested_wilson_equals_plain_when_converged():
    wl = workload(1)
    op = WilsonOperator(wl.dims, wl.mass, wl.mu)
    plain = GR.forward(op, wl.links(), wl.psi(), wl.k)
    nested = N.nested_tsl_wilson(op, wl.links(), wl.psi(), wl.k, 56)
    assert nested["k_used"] == plain["k_used"]
    assert np.linalg.norm(nested["y"] - plain["y"]) / np.linalg.norm(plain["y"]) < 1e-9
    coarse = N.nested_tsl_wilson(op, wl.links(), wl.psi(), wl.k, 12)
    assert np.linalg.norm(coarse["y"] - plain["y"]) / np.linalg.norm(plain["y"]) > 1e-8
