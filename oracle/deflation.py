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


# ----------------------------------------------------------------------------------------
# derivative of the deflated sign function (Sec. 3 with App. E's eigenpair motion)
# ----------------------------------------------------------------------------------------
#
# S(U) = Re eta^H [ sum_i s_i Pi_i psi + TSL_k(H, (1 - sum_i Pi_i) psi) ],  Pi_i = R_i L_i^H,
# with the eigenpairs functions of U and s_i = sgn Re lambda_i (locally constant).
# For a simple eigenvalue the spectral projector moves as
#     dPi_i = Z_i dH Pi_i + Pi_i dH Z_i,   Z_i = (lambda_i - H)^{-1} (1 - Pi_i)
# (the reduced resolvent; residue of the resolvent's first-order perturbation).  With
# psibar_p = dS/dpsi_p of the TSL part and a_i = s_i eta - psibar_p,
#     dS = Re tr(G_TSL^H dU) + Re sum_i a_i^H dPi_i psi
#        = Re tr(G_TSL^H dU) + Re sum_i [ c_i (Z_i^H a_i)^H dH R_i + (a_i^H R_i) L_i^H dH (Z_i psi) ],
# c_i = L_i^H psi: rank-one terms Re x^H dH y contracted onto the links.

def reduced_resolvents(H: np.ndarray, idx):
    """Z_i = sum_{j != i} R_j L_j^H / (lambda_i - lambda_j) for the eigenpairs idx of the
    full spectrum (plain definition on tiny lattices).  Returns a list of n x n matrices
    and the full (lam, R, L) it used."""
    n = H.shape[0]
    lam, R, L = eigenpairs(H, n)
    out = []
    for i in idx:
        w = np.array([0.0 if j == i else 1.0 / (lam[i] - lam[j]) for j in range(n)], dtype=np.complex128)
        out.append((R * w[None, :]) @ L.conj().T)
    return out, (lam, R, L)


def deflated_objective(U, psi, eta, k, dims, mass, mu, l, **kw) -> float:
    """S with the l smallest-|lambda| eigenpairs recomputed from U (finite differences)."""
    from .wilson import WilsonOperator, dense_h
    H = dense_h(U, dims, mass, mu)
    lam, R, L = eigenpairs(H, l)
    op = WilsonOperator(dims, mass, mu)
    y = deflated_sign(op, U, psi, k, lam, R, L, **kw)
    return float(np.real(np.vdot(eta.ravel(), y.ravel())))


def deflated_gradient(U, psi, eta, k, dims, mass, mu, l, **kw):
    """(G, S, psibar) of the deflated S over all links, eigenpair motion included.

    The TSL part is differentiated by torch autograd through the oracle TSL
    (link gradient and source gradient); the eigenpair part uses the reduced
    resolvents of the full dense spectrum.  With l = n the complement is empty
    and S is the exact Re eta^H sgn(H) psi.
    """
    from .grad import grad_autograd, link_gradient_from_matrix
    from .wilson import WilsonOperator, dense_h
    op = WilsonOperator(dims, mass, mu)
    H = dense_h(U, dims, mass, mu)
    n = H.shape[0]
    lam, R, L = eigenpairs(H, l)
    x, e = psi.ravel(), eta.ravel()
    c = L.conj().T @ x
    xp = x - R @ c
    s = np.sign(lam.real)
    if l < n:
        g = grad_autograd(op, U, xp.reshape(psi.shape), eta, k, **kw)
        G, S, pbar = g["G"], g["S"], g["dpsi"].ravel()
    else:
        G, S, pbar = np.zeros((4, op.volume, 3, 3), dtype=np.complex128), 0.0, np.zeros(n, dtype=np.complex128)
    S += float(np.real(np.vdot(e, R @ (s * c))))
    Zs, _ = reduced_resolvents(H, range(l))
    Gam = np.zeros((n, n), dtype=np.complex128)
    for i in range(l):
        a = s[i] * e - pbar
        x1 = np.conj(c[i]) * (Zs[i].conj().T @ a)          # Re x1^H dH R_i
        x2 = np.vdot(R[:, i], a) * L[:, i]                   # (R_i^H a) L_i:  Re x2^H dH (Z_i psi)
        Gam += np.outer(R[:, i], x1.conj()) + np.outer(Zs[i] @ x, x2.conj())
    G = G + link_gradient_from_matrix(Gam, U, op)
    # source gradient: S = Re eta^H sum_i s_i R_i L_i^H psi + S_TSL((1 - R L^H) psi)
    pb = L @ (s * (R.conj().T @ e)) + pbar - L @ (R.conj().T @ pbar)
    return G, S, pb.reshape(psi.shape)
