"""Oracle U(1) link-current trace estimator (Sec. 4, divergence of the U(1) vector current).

Test infrastructure only: imported by tests and benchmarks, never by the library.

The link current of eq. lat_vec_cur is a trace over the derivative of the overlap
operator with respect to the Abelian link phase Theta_{x,nu} (U_nu(x) -> e^{i Theta} U_nu(x)).
Without the inverse Dirac operator (not part of this path) the trace that the
sign-function derivative gives is

    j(x, nu) = Re Tr( dD_ov / dTheta_{x,nu} ) = Re Tr( g5 d sgn(H) / dTheta_{x,nu} ),

because D_ov = 1 + g5 sgn(H) (eq. overlap, a = 1).  The stochastic estimator with
Z2 noise xi_s (the paper's choice) is

    j_N(x, nu) = (1/N) sum_s d/dTheta_{x,nu} Re <g5 xi_s | sgn(H) | xi_s>,

each term the U(1) projection -Im tr(G_s^H U_nu(x)) of the link gradient G_s of
S_s = Re <eta_s | sgn(H) | psi_s> with eta_s = g5 xi_s, psi_s = xi_s.  Gauge
invariance of Tr(g5 sgn H) makes the divergence of eq. divergence_def,
div(x) = sum_nu [j(x, nu) - j(x - nu, nu)], vanish for the exact trace; the
"total current" flips the sign of the incoming term.  For a single noise sample
the divergence equals the source terms of the Ward identity in oracle.grad.

Functions:
* ``current_tsl``     -- the estimator with sgn(H) replaced by TSL_k per source
                         (torch autograd through the oracle TSL);
* ``exact_current``   -- Re Tr(A^H-weighted) derivative with the exact sign on tiny
                         lattices: Daleckii-Krein with the matrix A in place of
                         psi eta^H (A = g5 for the full trace, A = (1/N) sum xi (g5 xi)^H
                         for the estimator with the exact sign);
* ``divergence``      -- divergence and total current of eq. divergence_def;
* ``physical_current`` -- the current of eq. lat_vec_cur itself,
                         j = Tr(D_ov^{-1} dD_ov/dTheta) (complex), exactly (dense D_ov
                         with the Schur sign, tiny lattices) or as the Z2-noise
                         estimator (1/N) sum_s xi_s^H D_ov^{-1} dD_ov/dTheta xi_s with the
                         same exact operators.  With A fixed, Tr(A g5 d sgn(H)) is the
                         derivative of tr(A g5 sgn(H)) at fixed A, so both forms are
                         ``exact_current`` with A = D_ov^{-1} g5 (resp. the noise
                         average of xi xi^H D_ov^{-1} g5) for the real part and -i A for
                         the imaginary part.
"""
from __future__ import annotations

import numpy as np

from .grad import grad_autograd, link_gradient_from_matrix, u1_projection
from .sign import daleckii_krein, sign_schur
from .wilson import WilsonOperator, dense_h, gamma5


def g5_source(xi: np.ndarray) -> np.ndarray:
    """g5 xi for a canonical spinor (V, 4, 3)."""
    return xi * np.diag(gamma5()).real[None, :, None]


def current_tsl(op: WilsonOperator, U: np.ndarray, xis: np.ndarray, ks, **kw):
    """Estimator j_N (4, V) with TSL_{k_s} per source, and the per-source gradients."""
    per = []
    j = np.zeros((4, op.volume))
    for xi, k in zip(xis, ks):
        r = grad_autograd(op, U, xi, g5_source(xi), int(k), **kw)
        per.append(r)
        j += u1_projection(r["G"], U)
    return j / len(per), per


def exact_current(U: np.ndarray, dims, mass: float, mu: float, A: np.ndarray | None = None) -> np.ndarray:
    """d/dTheta_{x,nu} Re tr(A sgn(H)) for all links (tiny lattices); A = g5 by default.

    Re tr(A sgn(H)) generalises Re eta^H sgn(H) psi = Re tr(psi eta^H sgn(H)), so the
    Daleckii-Krein gradient matrix is taken with A in place of psi eta^H.
    """
    op = WilsonOperator(dims, mass, mu)
    n = 12 * op.volume
    if A is None:
        A = np.diag(np.tile(np.repeat(np.diag(gamma5()).real, 3), op.volume)).astype(np.complex128)
    assert A.shape == (n, n)
    H = dense_h(U, dims, mass, mu)
    G = link_gradient_from_matrix(daleckii_krein(H, A), U, op)
    return u1_projection(G, U)


def divergence(j: np.ndarray, op: WilsonOperator):
    """(div, tot) per site: sum_nu [j(x, nu) -+ j(x - nu, nu)]."""
    bwd = op.geom.bwd
    div = sum(j[nu] - j[nu][bwd[nu]] for nu in range(4))
    tot = sum(j[nu] + j[nu][bwd[nu]] for nu in range(4))
    return div, tot


def overlap_dense(U: np.ndarray, dims, mass: float, mu: float) -> np.ndarray:
    """D_ov = 1 + g5 sgn(H) (eq. overlap, a = 1) with the Schur sign (tiny lattices)."""
    H = dense_h(U, dims, mass, mu)
    g5 = np.tile(np.repeat(np.diag(gamma5()).real, 3), H.shape[0] // 12)
    return np.eye(H.shape[0], dtype=np.complex128) + g5[:, None] * sign_schur(H)


def physical_current(U: np.ndarray, dims, mass: float, mu: float, xis: np.ndarray | None = None) -> np.ndarray:
    """j(x, nu) = Tr(D_ov^{-1} dD_ov/dTheta_{x,nu}) as complex (4, V); with noise vectors
    xis (N, V, 4, 3) the estimator (1/N) sum_s xi_s^H D_ov^{-1} dD_ov/dTheta xi_s."""
    n = 12 * int(np.prod(dims))
    Dinv = np.linalg.inv(overlap_dense(U, dims, mass, mu))
    g5 = np.tile(np.repeat(np.diag(gamma5()).real, 3), n // 12)
    W = Dinv * g5[None, :]                           # D_ov^{-1} g5
    if xis is not None:
        X = xis.reshape(len(xis), n).T               # columns xi_s
        W = (X @ (X.conj().T @ W)) / len(xis)        # (1/N) sum xi xi^H D^{-1} g5
    return exact_current(U, dims, mass, mu, W) + 1j * exact_current(U, dims, mass, mu, -1j * W)


def current_deflated(U: np.ndarray, xis: np.ndarray, ks, dims, mass: float, mu: float, l: int, **kw):
    """Estimator j_N (4, V) with the deflated TSL sign per source (Sec. 4.3 with Sec. 3):
    each term the U(1) projection of the deflated link gradient (the eigenpairs' motion
    included) of Re <g5 xi_s | sgn(H) | xi_s>, the l smallest-|lambda| eigenpairs of the
    dense H deflated.  With l = n the sign is exact and so is each term."""
    from .deflation import deflated_gradient
    j = np.zeros((4, int(np.prod(dims))))
    for xi, k in zip(xis, ks):
        G, _, _ = deflated_gradient(U, xi, g5_source(xi), int(k), dims, mass, mu, l, **kw)
        j += u1_projection(G, U)
    return j / len(xis)
