"""Oracle of the paper's own derivative method (Sec. 2, Theorem 1, eq. func_derivative_1)
and its error estimate (Sec. 4.1, eq. bA_error_est).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a matrix A(t), Theorem 1 puts the derivative into the block matrix
B = [[A, dA], [0, A]]:  f(B) = [[f(A), d f(A)], [0, f(A)]], so that
f(B) (0, x) = (d f(A) x, f(A) x).  The method approximates f(B) (0, x) by the same
two-sided Lanczos process as f(A) x, now on vectors of length 2n (both Krylov
spaces of B started from the source), and reads the derivative off the upper half.
Here A = H(mu) = g5 D_w(mu) and t is the parameter of one link,
U_nu(site) -> exp(i t X) U_nu(site); dH is linear in U, so dH v is H evaluated on a
gauge field that is zero except for the one link i X U_nu(site), minus g5 v (the
diagonal part of H).  Its adjoint is the same construction with -mu (H^dag = H(-mu)).

Deflation of the block process (App. E) treats the invariant subspace of B belonging to
the l smallest-|lambda| eigenpairs of A exactly (deflated_block_sign below).

The error estimate of eq. bA_error_est applies the approximation twice:
eps_B = |TSL(B, TSL(B, (0, psi))) - (0, psi)| / (2 |psi|), the second process a fresh
one whose source is the first result (both of its Krylov spaces started there).
"""
from __future__ import annotations

import numpy as np
import torch

from .deflation import eigenpairs
from .tsl import tsl


def link_direction_field(U: np.ndarray, nu: int, site: int, X: np.ndarray) -> np.ndarray:
    """The gauge field dU of the link tangent: zero except dU_nu(site) = i X U_nu(site)."""
    dU = np.zeros_like(U)
    dU[nu, site] = 1j * np.asarray(X) @ U[nu, site]
    return dU


class BlockOperator:
    """B = [[H, dH], [0, H]] and B^H = [[H^H, 0], [dH^H, H^H]] on flat 2n vectors."""

    def __init__(self, op, U: np.ndarray, dU: np.ndarray, shape):
        self.op = op
        self.U = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128))
        self.dU = torch.from_numpy(np.ascontiguousarray(dU, dtype=np.complex128))
        self.zero = torch.zeros_like(self.U)
        self.shape = shape
        self.n = int(np.prod(shape))

    def dh(self, v):
        return (self.op.h(self.dU, v.view(self.shape)) - self.op.h(self.zero, v.view(self.shape))).reshape(-1)

    def dh_dag(self, v):
        return (self.op.h_dag(self.dU, v.view(self.shape)) - self.op.h_dag(self.zero, v.view(self.shape))).reshape(-1)

    def h(self, v):
        return self.op.h(self.U, v.view(self.shape)).reshape(-1)

    def h_dag(self, v):
        return self.op.h_dag(self.U, v.view(self.shape)).reshape(-1)

    def apply(self, z):
        z1, z2 = z[:self.n], z[self.n:]
        return torch.cat([self.h(z1) + self.dh(z2), self.h(z2)])

    def apply_dag(self, z):
        z1, z2 = z[:self.n], z[self.n:]
        return torch.cat([self.h_dag(z1), self.dh_dag(z1) + self.h_dag(z2)])


def block_tsl(bop: BlockOperator, x1: np.ndarray, x2: np.ndarray, k: int, **kw):
    """TSL_k(B, (x1, x2)): dict with the upper and lower halves of the result, T and k_used."""
    x = torch.from_numpy(np.concatenate([np.ravel(x1), np.ravel(x2)]).astype(np.complex128))
    with torch.no_grad():
        res = tsl(bop.apply, bop.apply_dag, x, k, **kw)
    y = res.y.numpy()
    return dict(y1=y[:bop.n].reshape(bop.shape), y2=y[bop.n:].reshape(bop.shape), T=res.T.numpy(),
                k_used=res.k_used, breakdown=res.breakdown)


def d1_derivative(op, U: np.ndarray, psi: np.ndarray, k: int, nu: int, site: int, X: np.ndarray, **kw):
    """The paper's derivative of sgn(H) psi along U_nu(site) -> exp(i t X) U_nu(site):
    the upper half of TSL_k(B, (0, psi)) (and the lower half, the sign itself)."""
    bop = BlockOperator(op, U, link_direction_field(U, nu, site, X), psi.shape)
    return block_tsl(bop, np.zeros_like(psi), psi, k, **kw)


def eps_block(op, U: np.ndarray, psi: np.ndarray, k: int, nu: int, site: int, X: np.ndarray, **kw) -> float:
    """eps_B of eq. bA_error_est for the same direction and Krylov size."""
    bop = BlockOperator(op, U, link_direction_field(U, nu, site, X), psi.shape)
    first = block_tsl(bop, np.zeros_like(psi), psi, k, **kw)
    second = block_tsl(bop, first["y1"], first["y2"], k, **kw)
    diff = np.concatenate([second["y1"].ravel(), (second["y2"] - psi).ravel()])
    return float(np.linalg.norm(diff) / (2.0 * np.linalg.norm(psi)))


def frozen_polynomial_derivative(A: np.ndarray, dA: np.ndarray, x: np.ndarray, ritz: np.ndarray) -> np.ndarray:
    """d/dt p(A + t dA) x at t = 0 for the polynomial p of degree k-1 that interpolates
    sgn(Re z) at the Ritz values (Newton form, product rule; no Lanczos vectors).  The
    nodes are taken in Leja order (each next node farthest, in the product of
    distances, from those before it), which keeps the divided differences stable;
    the interpolating polynomial itself does not depend on the order."""
    th0 = list(np.asarray(ritz, dtype=np.complex128))
    order = [int(np.argmax(np.abs(th0)))]
    while len(order) < len(th0):
        rest = [i for i in range(len(th0)) if i not in order]
        logd = [sum(np.log(abs(th0[i] - th0[j]) + 1e-300) for j in order) for i in rest]
        order.append(rest[int(np.argmax(logd))])
    th = np.asarray([th0[i] for i in order])
    f = np.sign(th.real).astype(np.complex128)
    k = len(th)
    coef = f.copy()
    for lev in range(1, k):
        coef[lev:] = (coef[lev:] - coef[lev - 1:-1]) / (th[lev:] - th[:k - lev])
    prod, dprod = x.astype(np.complex128), np.zeros_like(x, dtype=np.complex128)
    out = np.zeros_like(dprod)
    for i in range(1, k):
        dprod = dA @ prod + A @ dprod - th[i - 1] * dprod
        prod = A @ prod - th[i - 1] * prod
        out = out + coef[i] * dprod
    return out


# ----------------------------------------------------------------------------------------
# deflation of the block-matrix process (App. E, eq. array_app_defl_1 and its coefficients)
# ----------------------------------------------------------------------------------------
#
# For B = [[A, dA], [0, A]] the deflated eigenpairs (lambda_i, R_i, L_i) of A, L^H R = I,
# span a 2l-dimensional invariant subspace of B with right basis (R_i, 0), (dR_i, R_i)
# and left basis (L_i, dL_i), (0, L_i).  With s_i = sgn Re lambda_i (locally constant),
#     sgn(B) x = sum_i s_i [ (R_i, 0) c1_i + (dR_i, R_i) c2_i ] + sgn(B) Pbar x,
#     c2_i = <L_i|x2>,   c1_i = <L_i|x1> + <dL_i|x2>,
#     Pbar x = (x1 - sum_i (c1_i R_i + c2_i dR_i), x2 - sum_i c2_i R_i),
# and sgn(B) Pbar x is left to the TSL process on B.  The eigenvector derivatives are
# normalised with <dL_i|R_i> = <L_i|dR_i> = 0:
#     dR_i = sum_{j != i} R_j (L_j^H dA R_i) / (lambda_i - lambda_j),
#     <dL_i|x> = sum_{j != i} (L_i^H dA R_j) (L_j^H x) / (lambda_i - lambda_j),
# the sums over the whole spectrum (here from the dense eigendecomposition).  Every
# coefficient is taken from the input (x1, x2), so that Pbar x has no component along
# the deflated subspace; (App. E's listing instead subtracts each pair's part from x1
# before forming the next c1, which would leave -sum_{j<i} c2_j <L_i|dR_j> in c1_i.)

def eigenvector_derivatives(H: np.ndarray, dH: np.ndarray, l: int):
    """(lam, R, L, dR, dLx) for the l smallest-|lambda| eigenpairs of the dense H moving
    with dH: dR (n, l) the right eigenvector derivatives and dLx(x) -> (l,) the values
    <dL_i|x>, both from the full dense eigendecomposition."""
    n = H.shape[0]
    lam_all, R_all, L_all = eigenpairs(H, n)
    lam, R, L = lam_all[:l], R_all[:, :l], L_all[:, :l]
    M = L_all.conj().T @ dH @ R_all          # M[j, i] = L_j^H dA R_i
    diff = lam_all[:l][:, None] - lam_all[None, :]   # [i, j] = lambda_i - lambda_j
    W = np.zeros((l, n), dtype=np.complex128)
    for i in range(l):
        for j in range(n):
            if j != i:
                W[i, j] = 1.0 / diff[i, j]
    dR = np.zeros((n, l), dtype=np.complex128)
    for i in range(l):
        dR[:, i] = R_all @ (M[:, i] * W[i])

    def dLx(x):
        c = L_all.conj().T @ x               # L_j^H x over the whole spectrum
        return np.array([np.sum(M[i, :] * c * W[i]) for i in range(l)])

    return lam, R, L, dR, dLx


def deflated_block_sign(op, U: np.ndarray, dU: np.ndarray, x1: np.ndarray, x2: np.ndarray, k: int, l: int,
                        dims, mass, mu, **kw):
    """sgn(B)(x1, x2) with the l smallest-|lambda| eigenpairs of A = H deflated: the exact
    part of eq. array_app_defl_1 plus TSL_k(B, Pbar x).  Returns y1, y2 (canonical) and
    the projected source with its coefficients (for the pins)."""
    from .wilson import dense_h
    H = dense_h(U, dims, mass, mu)
    dH = dense_h(U + dU, dims, mass, mu) - H       # H is affine in U
    lam, R, L, dR, dLx = eigenvector_derivatives(H, dH, l)
    a, b = np.ravel(x1).astype(np.complex128), np.ravel(x2).astype(np.complex128)
    c2 = L.conj().T @ b
    c1 = L.conj().T @ a + dLx(b)
    s = np.sign(lam.real)
    out1 = R @ (s * c1) + dR @ (s * c2)
    out2 = R @ (s * c2)
    p1 = a - R @ c1 - dR @ c2
    p2 = b - R @ c2
    shape = np.shape(x2)
    if np.linalg.norm(np.concatenate([p1, p2])) > 0.0:
        bop = BlockOperator(op, U, dU, shape)
        res = block_tsl(bop, p1.reshape(shape), p2.reshape(shape), k, **kw)
        out1 = out1 + res["y1"].ravel()
        out2 = out2 + res["y2"].ravel()
    return dict(y1=out1.reshape(shape), y2=out2.reshape(shape), p1=p1, p2=p2, c1=c1, c2=c2,
                lam=lam, R=R, L=L, dR=dR, H=H, dH=dH)


def eps_block_deflated(op, U, dU, psi, k, l, dims, mass, mu, **kw) -> float:
    """eps_B of eq. bA_error_est with the deflated block sign applied twice (App. E's
    reason for deflating general sources)."""
    first = deflated_block_sign(op, U, dU, np.zeros_like(psi), psi, k, l, dims, mass, mu, **kw)
    second = deflated_block_sign(op, U, dU, first["y1"], first["y2"], k, l, dims, mass, mu, **kw)
    diff = np.concatenate([second["y1"].ravel(), (second["y2"] - psi).ravel()])
    return float(np.linalg.norm(diff) / (2.0 * np.linalg.norm(psi)))
