"""Oracle matrix sign function and its Frechet derivative (Sec. 2).

The matrix sign function of a diagonalisable A = X diag(l_i) X^{-1} is
X diag(sgn Re l_i) X^{-1} (eq. spectral_form and the remark after it); it is
undefined when an eigenvalue lies on Re z = 0.  Three independent evaluations:

* ``sign_schur``  -- complex Schur form reordered so that the right-half-plane
  eigenvalues come first; then sgn = Q [[I, X], [0, -I]] Q^H where X solves the
  Sylvester equation T11 X - X T22 = 2 T12 (sgn(T) commutes with T);
* ``sign_eig``    -- the spectral form itself;
* ``sign_newton`` -- Newton iteration S <- (S + S^{-1})/2 with determinant scaling.

``frechet_sign`` applies Theorem 1 (Mathias): the upper-right block of
sgn([[A, E], [0, A]]) is the Frechet derivative L_sgn(A, E), i.e. d/dt sgn(A + tE).
``daleckii_krein`` is the same derivative written in the eigenbasis (divided
differences of sgn), used as an independent check of Theorem 1 on small matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class SignUndefined(ValueError):
    """An eigenvalue lies on (or numerically on) the line Re z = 0."""


def _check_gap(eigs: np.ndarray, scale: float, tol: float = 1e-12):
    m = np.min(np.abs(eigs.real)) if eigs.size else np.inf
    if m <= tol * scale:
        raise SignUndefined(f"eigenvalue with |Re| = {m:.3e} on the sign discontinuity")
    return m


def sign_schur(A: np.ndarray) -> np.ndarray:
    """sgn(A) through the reordered complex Schur form and a Sylvester solve."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    T, Q, sdim = sla.schur(A, output="complex", sort="rhp")
    _check_gap(np.diag(T), max(np.abs(T).max(), 1e-300))
    S = np.zeros_like(T)
    S[:sdim, :sdim] = np.eye(sdim)
    S[sdim:, sdim:] = -np.eye(n - sdim)
    if 0 < sdim < n:
        S[:sdim, sdim:] = sla.solve_sylvester(T[:sdim, :sdim], -T[sdim:, sdim:], 2.0 * T[:sdim, sdim:])
    return Q @ S @ Q.conj().T


def sign_eig(A: np.ndarray) -> np.ndarray:
    """sgn(A) = X diag(sgn Re l_i) X^{-1} (eq. spectral_form)."""
    w, X = np.linalg.eig(np.asarray(A, dtype=np.complex128))
    _check_gap(w, max(np.abs(w).max(), 1e-300))
    return X @ np.diag(np.sign(w.real)) @ np.linalg.inv(X)


def sign_newton(A: np.ndarray, tol: float = 1e-14, maxit: int = 100) -> np.ndarray:
    """Scaled Newton iteration for sgn(A) (determinant scaling, switched off near convergence)."""
    S = np.asarray(A, dtype=np.complex128).copy()
    n = S.shape[0]
    scale_on = True
    for _ in range(maxit):
        Si = np.linalg.inv(S)
        if scale_on:
            _, logdet = np.linalg.slogdet(S)
            g = np.exp(-logdet / n)
        else:
            g = 1.0
        Sn = 0.5 * (g * S + Si / g)
        delta = np.linalg.norm(Sn - S) / np.linalg.norm(Sn)
        S = Sn
        if delta < 1e-2:
            scale_on = False
        if delta < tol:
            return S
    raise RuntimeError("Newton sign iteration did not converge")


def frechet_sign(A: np.ndarray, E: np.ndarray) -> np.ndarray:
    """L_sgn(A, E) as the upper-right block of sgn([[A, E], [0, A]]) (Theorem 1)."""
    n = A.shape[0]
    B = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    B[:n, :n] = A
    B[n:, n:] = A
    B[:n, n:] = E
    return sign_schur(B)[:n, n:]


def daleckii_krein(A: np.ndarray, E: np.ndarray) -> np.ndarray:
    """L_sgn(A, E) = X [F o (X^{-1} E X)] X^{-1}, F_ij = divided difference of sgn.

    F_ij = (s_i - s_j)/(l_i - l_j) and 0 where s_i = s_j (sgn is locally
    constant, so its derivative vanishes on the spectrum).
    """
    w, X = np.linalg.eig(np.asarray(A, dtype=np.complex128))
    s = np.sign(w.real)
    Xi = np.linalg.inv(X)
    diff = w[:, None] - w[None, :]
    same = s[:, None] == s[None, :]
    F = np.where(same, 0.0, (s[:, None] - s[None, :]) / np.where(same, 1.0, diff))
    return X @ (F * (Xi @ E @ X)) @ Xi
