"""Oracle derivative of S_k(U) = Re <eta | TSL_k(H(U), psi)> with respect to the links.

Conventions.  The gradient with respect to a link is the complex 3x3 matrix
G = dS/dRe U + i dS/dIm U, so that dS = Re tr(G^H dU).  The U(1) projection
(link phase U -> e^{i theta} U, the Abelian field Theta of eq. WD_G) is
dS/dtheta = -Im tr(G^H U); the su(3) direction U -> e^{i w X} U gives
dS/dw = -Im tr(G^H X U).

Derivative definition: the exact derivative of the k-step TSL scalar, i.e. the
derivative of eq. derivative_def taken through the approximation itself, with
the Frechet derivative of sgn on T_k by Theorem 1.  Computed here by torch
autograd through the plain oracle TSL (``grad_autograd``), by central finite
differences (``fd_directional``) and, for the exact sign function on tiny
lattices, by the Daleckii-Krein formula contracted onto the links
(``exact_gradient``).  ``ward_residual`` evaluates the U(1) gauge identity that
follows from gauge invariance of the operator (Sec. 4.3, eq. divergence_def):
at every site  sum_nu (g_{x,nu} - g_{x-nu,nu}) = -Im eta(x)^H y(x) + Im psibar(x)^H psi(x),
with g the U(1) projection of G and psibar = dS/dpsi.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import torch

from .sign import daleckii_krein, sign_schur
from .tsl import tsl_wilson
from .wilson import WilsonOperator, dense_h, gamma5, gamma_matrices


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))


def objective(op: WilsonOperator, U: torch.Tensor, psi: torch.Tensor, eta: torch.Tensor, k: int, **kw):
    """S_k = Re eta^H TSL_k(H(U), psi) and the TSL result (differentiable)."""
    res = tsl_wilson(op, U, psi, k, **kw)
    return torch.real(torch.sum(eta.conj() * res.y)), res


def grad_autograd(op: WilsonOperator, U: np.ndarray, psi: np.ndarray, eta: np.ndarray, k: int, **kw):
    """All-links gradient G (4, V, 3, 3), S, y, dS/dpsi and k_used by torch autograd."""
    Ut = _t(U).requires_grad_(True)
    pt = _t(psi).requires_grad_(True)
    S, res = objective(op, Ut, pt, _t(eta), k, **kw)
    S.backward()
    return dict(G=Ut.grad.numpy(), S=float(S.detach()), y=res.y.detach().numpy(), dpsi=pt.grad.numpy(),
                k_used=res.k_used, T=res.T.detach().numpy())


def forward(op: WilsonOperator, U: np.ndarray, psi: np.ndarray, k: int, **kw):
    """TSL_k(H(U), psi) without gradients: dict with y, T, c, k_used, breakdown, and
    biorth = |w_1^H v_k| + |w_k^H v_1| (k = k_used; 0 below 2), the entries of
    W^H V - I farthest from the diagonal under the normalisation w_j^H v_j = 1."""
    with torch.no_grad():
        res = tsl_wilson(op, _t(U), _t(psi), k, **kw)
        kk = res.k_used
        bi = 0.0
        if kk >= 2:
            bi = float(abs(torch.vdot(res.W[0], res.V[kk - 1])) + abs(torch.vdot(res.W[kk - 1], res.V[0])))
    return dict(y=res.y.numpy(), T=res.T.numpy(), c=res.c.numpy(), k_used=res.k_used,
                breakdown=res.breakdown, alpha=np.array([complex(a) for a in res.alpha]), biorth=bi)


def su3_direction(rng: np.random.Generator) -> np.ndarray:
    """Random Hermitian traceless 3x3 matrix of unit Frobenius norm."""
    a = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    h = a + a.conj().T
    h -= np.trace(h) / 3 * np.eye(3)
    return h / np.linalg.norm(h)


def rotate_link(U: np.ndarray, nu: int, site: int, X: np.ndarray, h: float) -> np.ndarray:
    """Copy of U with U_nu(site) -> exp(i h X) U_nu(site)."""
    Up = U.copy()
    Up[nu, site] = sla.expm(1j * h * X) @ U[nu, site]
    return Up


def fd_directional(S_of_U, U: np.ndarray, nu: int, site: int, X: np.ndarray, h: float = 1e-5) -> float:
    """Central difference of S along U_nu(site) -> exp(i h X) U_nu(site)."""
    return (S_of_U(rotate_link(U, nu, site, X, h)) - S_of_U(rotate_link(U, nu, site, X, -h))) / (2 * h)


def directional_from_gradient(G: np.ndarray, U: np.ndarray, nu: int, site: int, X: np.ndarray) -> float:
    """dS/dw for U_nu(site) -> exp(i w X) U_nu(site):  -Im tr(G^H X U)."""
    return float(-np.imag(np.trace(G[nu, site].conj().T @ X @ U[nu, site])))


def u1_projection(G: np.ndarray, U: np.ndarray) -> np.ndarray:
    """g_{x,nu} = dS/dtheta_{x,nu} = -Im tr(G^H U), shape (4, V)."""
    return -np.imag(np.einsum("nvab,nvab->nv", G.conj(), U))


def ward_residual(op: WilsonOperator, G, U, psi, eta, y, dpsi) -> tuple[np.ndarray, np.ndarray]:
    """(lhs, rhs) per site of the U(1) Ward identity stated in the module docstring."""
    g = u1_projection(G, U)
    bwd = op.geom.bwd
    lhs = sum(g[nu] - g[nu][bwd[nu]] for nu in range(4))
    rhs = -np.imag(np.einsum("vsa,vsa->v", eta.conj(), y)) + np.imag(np.einsum("vsa,vsa->v", dpsi.conj(), psi))
    return lhs, rhs


# ----------------------------------------------------------------------------------------
# exact sign function on tiny lattices
# ----------------------------------------------------------------------------------------

def exact_objective(U, psi, eta, dims, mass, mu) -> float:
    """Re eta^H sgn(H) psi with the dense Schur sign (tiny lattices)."""
    H = dense_h(U, dims, mass, mu)
    return float(np.real(np.vdot(eta.ravel(), sign_schur(H) @ psi.ravel())))


def link_gradient_from_matrix(Gam: np.ndarray, U: np.ndarray, op: WilsonOperator) -> np.ndarray:
    """Contract dS = Re tr(dH Gam) onto the links (dense Gam, tiny lattices).

    For the forward hop at x (block row x, column x+nu) dD = c_f (1+g_nu) (x) dU and
    for the backward hop at x+nu (block row x+nu, column x) dD = c_b (1-g_nu) (x) dU^H,
    with c_f = -kappa e^{+mu d} sigma and c_b = -kappa e^{-mu d} sigma (sigma the
    boundary sign).  Since H = g5 D_w, dS = Re tr(g5 dD Gam), and collecting the
    coefficient of dU gives G = c_f conj(M1) + c_b M2^T with
    M1_ab = sum_st (g5)_s (1+g)_st Gam[(x+nu,t,b),(x,s,a)] and
    M2_ab = sum_st (g5)_s (1-g)_st Gam[(x,t,b),(x+nu,s,a)].
    """
    V = op.volume
    gam = gamma_matrices()
    g5 = np.diag(gamma5()).real
    Gm = Gam.reshape(V, 4, 3, V, 4, 3)
    out = np.zeros((4, V, 3, 3), dtype=np.complex128)
    one = np.eye(4)
    for nu in range(4):
        e = math.exp(op.mu) if nu == 3 else 1.0
        for x in range(V):
            y = op.geom.fwd[nu, x]
            sig = op.geom.sign_fwd[nu, x]
            pf = g5[:, None] * (one + gam[nu])
            pb = g5[:, None] * (one - gam[nu])
            M1 = np.einsum("st,tbsa->ab", pf, Gm[y, :, :, x, :, :])
            M2 = np.einsum("st,tbsa->ab", pb, Gm[x, :, :, y, :, :])
            out[nu, x] = -op.kappa * sig * (e * M1.conj() + M2.T / e)
    return out


def exact_gradient(U, psi, eta, dims, mass, mu) -> np.ndarray:
    """Gradient of Re eta^H sgn(H) psi over all links by Daleckii-Krein (tiny lattices).

    dS = Re eta^H L(H, dH) psi = Re tr(dH L(H, psi eta^H)) by the trace
    identity of Frechet derivatives of primary matrix functions.
    """
    op = WilsonOperator(dims, mass, mu)
    H = dense_h(U, dims, mass, mu)
    Gam = daleckii_krein(H, np.outer(psi.ravel(), eta.ravel().conj()))
    return link_gradient_from_matrix(Gam, U, op)
