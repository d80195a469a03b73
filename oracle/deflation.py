"""Oracle deflated sign function and error estimate (Sec. 3, Sec. 4.1).

For a diagonalisable H with right/left eigenvectors R_i, L_i normalised so that
L_i^H R_j = delta_ij (App. B, eq. eignorm), the l deflated eigenpairs are treated
exactly and the remainder by TSL (Sec. 3, eq. final_res; for the sign function
itself -- no block matrix -- there is no mixing term):

    c = L^H psi,   psi_p = psi - R c,   sgn(H) psi ~ TSL_k(H, psi_p) + R diag(sgn Re lambda) c.

The eigenpairs are the l smallest in |lambda| (the choice the paper uses for the
sign function).  The error estimate applies TSL twice (Sec. 4.1, eq. error_est):
eps_A = |TSL(TSL(psi)) - psi| / (2 |psi|), the second TSL a fresh Krylov space
with the first result as its source.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import torch

from .tsl import tsl_wilson


def eigenpairs(H: np.ndarray, l: int):
    """l eigenpairs of smallest |lambda|: (lam, R, L) with R, L of shape (n, l), L^H R = I."""
    w, vl, vr = sla.eig(H, left=True, right=True)
    order = np.argsort(np.abs(w))[:l]
    lam = w[order]
    R = vr[:, order]
    L = vl[:, order]
    d = np.einsum("ni,ni->i", L.conj(), R)     # L_i^H R_i
    L = L / d.conj()[None, :]
    return lam, R, L


def deflated_sign(op, U: np.ndarray, psi: np.ndarray, k: int, lam, R, L, **kw):
    """Deflated TSL sgn(H) psi (canonical (V, 4, 3) in and out)."""
    x = psi.ravel()
    c = L.conj().T @ x
    xp = x - R @ c
    sgn = np.sign(np.real(lam))
    with torch.no_grad():
        if np.linalg.norm(xp) == 0.0:
            yp = np.zeros_like(xp)
        else:
            yp = tsl_wilson(op, torch.from_numpy(U), torch.from_numpy(xp.reshape(psi.shape)), k, **kw).y.numpy().ravel()
    return (yp + R @ (sgn * c)).reshape(psi.shape)


def error_estimate(sign_fn, psi: np.ndarray) -> float:
    """eps_A = |sgn(sgn(psi)) - psi| / (2 |psi|) for a sign approximation ``sign_fn``."""
    y = sign_fn(psi)
    z = sign_fn(y)
    return float(np.linalg.norm((z - psi).ravel()) / (2.0 * np.linalg.norm(psi.ravel())))
