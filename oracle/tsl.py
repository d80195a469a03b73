"""Oracle two-sided Lanczos (TSL) approximation of f(A) x for non-Hermitian A.

The paper cites the TSL algorithm without printing it (Sec. 1, Sec. 2: the
Krylov spaces of A and A^dagger built from the same source x).  The plain
method, as read here:

* v_1 = w_1 = x / |x|;
* for j = 1..k:  a = A v_j,  alpha_j = w_j^H a;
  r = a - alpha_j v_j - gamma_j v_{j-1},  s = A^H w_j - conj(alpha_j) w_j - beta_j w_{j-1};
  omega = s^H r,  beta_{j+1} = |omega|^{1/2},  gamma_{j+1} = omega / beta_{j+1};
  v_{j+1} = r / beta_{j+1},  w_{j+1} = s / conj(gamma_{j+1})   (so w_i^H v_j = delta_ij);
* T_k is tridiagonal with diagonal alpha, sub-diagonal beta_{j+1} and
  super-diagonal gamma_{j+1};  f(A) x ~ |x| V_k f(T_k) e_1.

k counts basis vectors (= applications of A); the implied polynomial has
degree k-1.  No re-biorthogonalisation unless ``reorth=True`` (used only by
the k = n pins).  Breakdown: "lucky" when the right residual r vanishes
relative to A v_j -- then K_j(A, x) is invariant, A V_j = V_j T_j, and
|x| V_j f(T_j) e_1 equals f(A) x exactly; "serious" when omega = s^H r
vanishes relative to |r| |s| otherwise (this includes s = 0 with r != 0).

All arithmetic is complex128 torch on the CPU, so the whole recursion is
differentiable by torch autograd.  The sign of T_k is evaluated by the Schur
method; its backward pass is Theorem 1 applied to the 2k x 2k block matrix.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .sign import frechet_sign, sign_schur

TAU_LUCKY = 1e-11
TAU_SERIOUS = 1e-14


class SeriousBreakdown(RuntimeError):
    pass


class SignMatrix(torch.autograd.Function):
    """sgn(T) for a small dense complex matrix; backward by Theorem 1.

    With dL = Re tr(G^H dS) and dS = L(T, dT):  dL = Re tr(dT L(T, G^H)),
    hence the adjoint of T is L(T, G^H)^H, the upper-right block of
    sgn([[T, G^H], [0, T]]) conjugate-transposed.
    """

    @staticmethod
    def forward(ctx, T):
        ctx.save_for_backward(T)
        return torch.from_numpy(sign_schur(T.detach().numpy()))

    @staticmethod
    def backward(ctx, grad):
        (T,) = ctx.saved_tensors
        L = frechet_sign(T.detach().numpy(), grad.detach().numpy().conj().T)
        return torch.from_numpy(L.conj().T.copy())


def sign_matrix(T: torch.Tensor) -> torch.Tensor:
    return SignMatrix.apply(T)


def make_dot(perm: np.ndarray | None = None):
    """Inner product a^H b; with ``perm`` the terms are summed in a permuted order."""
    if perm is None:
        return lambda a, b: torch.sum(a.conj() * b)
    p = torch.from_numpy(np.asarray(perm))
    return lambda a, b: torch.sum((a.conj() * b)[p])


@dataclass
class TSLResult:
    y: torch.Tensor          # |x| V_k f(T_k) e_1
    T: torch.Tensor          # k_used x k_used tridiagonal
    c: torch.Tensor          # f(T_k) e_1
    V: list                  # right Lanczos vectors v_1..v_k
    W: list                  # left Lanczos vectors w_1..w_k
    alpha: list
    beta: list               # beta_2..beta_k (real)
    gamma: list              # gamma_2..gamma_k
    norm_x: torch.Tensor
    k_used: int
    breakdown: int           # 0 none, 1 lucky


def tsl(apply_A, apply_Adag, x: torch.Tensor, k: int, *, f=sign_matrix, reorth: bool = False,
        perm=None, tau_lucky: float = TAU_LUCKY, tau_serious: float = TAU_SERIOUS) -> TSLResult:
    """Plain TSL on flat complex vectors; ``apply_A``/``apply_Adag`` act on flat vectors."""
    dot = make_dot(perm)
    nrm = lambda z: torch.sqrt(torch.real(dot(z, z)))  # noqa: E731
    norm_x = nrm(x)
    v = x / norm_x
    w = v
    V, W, alpha, beta, gamma = [v], [w], [], [], []
    v_prev = w_prev = None
    beta_j = gamma_j = None
    breakdown = 0
    for j in range(k):
        a = apply_A(v)
        al = dot(w, a)
        alpha.append(al)
        if j == k - 1:
            break
        b = apply_Adag(w)
        r = a - al * v
        s = b - al.conj() * w
        if v_prev is not None:
            r = r - gamma_j * v_prev
            s = s - beta_j * w_prev
        if reorth:
            for vi, wi in zip(V, W):
                r = r - vi * dot(wi, r)
                s = s - wi * dot(vi, s)
        om = dot(s, r)
        nr, ns = nrm(r), nrm(s)
        if float(nr.detach()) <= tau_lucky * float(nrm(a).detach()):
            breakdown = 1
            break
        omc = complex(om.detach())
        if not np.isfinite(omc) or abs(omc) <= tau_serious * float(nr.detach()) * float(ns.detach()):
            raise SeriousBreakdown(f"serious breakdown at j={j + 1}: |omega|={abs(omc):.3e}")
        be = torch.sqrt(torch.abs(om))
        ga = om / be
        v_prev, w_prev = v, w
        v = r / be
        w = s / ga.conj()
        beta_j, gamma_j = be, ga
        beta.append(be)
        gamma.append(ga)
        V.append(v)
        W.append(w)
    kk = len(alpha)
    T = torch.diag(torch.stack(alpha))
    if kk > 1:
        T = T + torch.diag(torch.stack(beta).to(torch.complex128), -1)
        T = T + torch.diag(torch.stack(gamma), 1)
    S = f(T)
    c = S[:, 0]
    y = norm_x * (torch.stack(V, dim=1) @ c)
    return TSLResult(y, T, c, V, W, alpha, beta, gamma, norm_x, kk, breakdown)


def tsl_wilson(op, U: torch.Tensor, psi: torch.Tensor, k: int, **kw) -> TSLResult:
    """TSL of sgn(H(mu)) psi with H = g5 D_w(mu) given by a ``WilsonOperator``."""
    shape = psi.shape
    A = lambda z: op.h(U, z.view(shape)).reshape(-1)        # noqa: E731
    Ad = lambda z: op.h_dag(U, z.view(shape)).reshape(-1)   # noqa: E731
    res = tsl(A, Ad, psi.reshape(-1), k, **kw)
    res.y = res.y.view(shape)
    return res


def tsl_dense(A: np.ndarray, x: np.ndarray, k: int, **kw) -> TSLResult:
    """TSL with an explicit matrix (small pins)."""
    At = torch.from_numpy(np.asarray(A, dtype=np.complex128))
    Ah = At.conj().T.contiguous()
    return tsl(lambda z: At @ z, lambda z: Ah @ z,
               torch.from_numpy(np.asarray(x, dtype=np.complex128)), k, **kw)


def ritz_interpolation(A: np.ndarray, x: np.ndarray, ritz: np.ndarray) -> np.ndarray:
    """p(A) x where p (degree k-1) interpolates sgn(Re z) at the k Ritz values.

    Newton divided differences on the distinct Ritz values, evaluated by
    Horner-like accumulation of (A - theta_i) products on the vector x.  This
    uses no Lanczos basis at all, so it checks the TSL result independently.
    """
    th = np.asarray(ritz, dtype=np.complex128)
    f = np.sign(th.real).astype(np.complex128)
    k = len(th)
    coef = f.copy()
    for lev in range(1, k):
        coef[lev:] = (coef[lev:] - coef[lev - 1:-1]) / (th[lev:] - th[:k - lev])
    out = coef[0] * x
    prod = x.copy()
    for i in range(1, k):
        prod = A @ prod - th[i - 1] * prod
        out = out + coef[i] * prod
    return out
