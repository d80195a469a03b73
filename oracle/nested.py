"""Oracle nested two-sided Lanczos: the projected-matrix step by an inner Krylov method.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes with one level of nesting and inner Krylov size 100 (Sec. 4.1,
first paragraph of the numerical setup) and cites the nested method without
describing it (Sec. 1).  Reading taken here: the outer TSL of size k^O gives the
tridiagonal T = T_{k^O} and the result |x| V sgn(T) e_1 (plain TSL, ``oracle.tsl``);
the nested method replaces the exact sgn(T) e_1 by a Krylov approximation of
size k^I, built for the inverse of the squared projected matrix:

    sgn(T) e_1 = T (T^2)^{-1/2} e_1 = T W^{1/2} e_1,   W = (T^2)^{-1},

and W^{1/2} e_1 is approximated by a two-sided Lanczos process on W with both
Krylov spaces started from e_1 (the same plain recursion as the outer one):
W^{1/2} e_1 ~ V' (T')^{1/2} e_1 with V' (k^O x k^I) and the inner projected
matrix T' (k^I x k^I), and the principal square root.  The identity holds since
z (z^2)^{-1/2} = sgn(Re z) for the principal branch.  Eigenvalues of T near zero
become the largest ones of W, the part of the spectrum Krylov spaces resolve
first, which is why the inner space can be small (this is our reading of the
"intermediate preconditioning" of the cited work).

With k^I >= k^O the inner space is the whole space and the result is the plain
TSL result; as k^I grows the inner result converges to sgn(T) e_1 (pinned in
tests/test_oracle_nested.py).  The inner square root is evaluated by SciPy's
Schur-based ``sqrtm``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import torch

from .tsl import tsl, tsl_dense


def inner_sign_e1(T: np.ndarray, k_inner: int):
    """Nested approximation of sgn(T) e_1: (c, inner k_used, inner T')."""
    T = np.asarray(T, dtype=np.complex128)
    k = T.shape[0]
    e1 = np.zeros(k, dtype=np.complex128)
    e1[0] = 1.0
    W = np.linalg.inv(T @ T)
    # the inner recursion with f = principal square root (its column 0 is used)
    res = tsl_dense(W, e1, min(k_inner, k), f=lambda M: torch.from_numpy(sla.sqrtm(M.detach().numpy())))
    u = res.y.numpy()                  # ~ W^{1/2} e_1 (|e_1| = 1)
    return T @ u, res.k_used, res.T.numpy()


def nested_matrix_function(k_inner: int):
    """A function f(T) for ``oracle.tsl.tsl`` whose column 0 is the nested sgn(T) e_1."""
    def f(T: torch.Tensor) -> torch.Tensor:
        Tn = T.detach().numpy()
        c, _, _ = inner_sign_e1(Tn, k_inner)
        out = np.zeros_like(Tn)
        out[:, 0] = c
        return torch.from_numpy(out)
    return f


def nested_tsl_wilson(op, U: np.ndarray, psi: np.ndarray, k_outer: int, k_inner: int, **kw):
    """y = |psi| V sgn_nested(T_{k_outer}) e_1 for H = g5 D_w(mu): dict with y, T, c, k_used."""
    shape = psi.shape
    Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128))
    A = lambda z: op.h(Ut, z.view(shape)).reshape(-1)        # noqa: E731
    Ad = lambda z: op.h_dag(Ut, z.view(shape)).reshape(-1)   # noqa: E731
    with torch.no_grad():
        res = tsl(A, Ad, torch.from_numpy(np.ascontiguousarray(psi, dtype=np.complex128)).reshape(-1), k_outer,
                  f=nested_matrix_function(k_inner), **kw)
    return dict(y=res.y.numpy().reshape(shape), T=res.T.numpy(), c=res.c.numpy(), k_used=res.k_used)
