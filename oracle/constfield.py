"""Exact eigenpairs of H(mu) for a gauge-rotated constant gauge field (closed form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The deflated method (Sec. 3, App. E) takes known eigenpairs of H as input, and the
derivative of the deflated sign function moves them with the links.  On random
SU(3) fields at the large workloads the near-zero spectrum is dense (a fixed
fraction of all 12 V eigenvalues lies below |lambda| = 0.1), so neither the
lowest eigenpairs nor the reduced-resolvent solves of the eigenpair motion are
resolvable there.  This module gives a field family whose every eigenpair is
known exactly at any volume:

    U_nu(x) = g(x) C_nu g(x + nu)^dag,

with four constant SU(3) matrices C_nu and any SU(3) field g(x).  H is gauge
covariant (App. A: with psi -> g psi the hop U_nu(x) psi(x + nu) becomes
g(x) C_nu psi(x + nu)), so its eigenvectors are g(x) times those of the constant
field.  The constant field is translation invariant: on a plane wave
e^{i p.x} chi, chi a 12-vector in spin x colour, it acts as the 12 x 12 matrix

    M(p) = g5 [1 - kappa sum_nu ( e^{+mu d_nu,t} e^{+i p_nu} (1 + g_nu) (x) C_nu
                                + e^{-mu d_nu,t} e^{-i p_nu} (1 - g_nu) (x) C_nu^dag )],

p_nu = 2 pi n / N_nu in space and p_t = pi (2n + 1) / N_t for antiperiodic time
(the boundary sign continues the wave).  Each momentum is a 12 x 12 eigenproblem
with right vectors u_k and left vectors w_k, w_k^H u_j = delta_kj, and

    R(x) = g(x) e^{i p.x} u_k / sqrt(V),   L(x) = g(x) e^{i p.x} w_k / sqrt(V)

(g acting on the colour index), so L^H R = 1 for the pair and 0 across
different (p, k).  When the C_nu commute (an abelian background) every
eigenvalue is doubly degenerate in spin (M^2 is then a scalar in spin); generic
non-commuting C_nu lift that, which the eigenpair motion needs.  Replacing C_nu by
exp(i t X_nu) C_nu keeps the field in the family, so the deflated function can be
differenced in t with exact eigenpairs on both sides; in terms of the links this
is U_nu(x) -> exp(i t g(x) X_nu g(x)^dag) U_nu(x).

Pinned by tests/test_oracle_constfield.py: the closed-form spectrum against the
dense eigenvalues of the oracle's dense H at 4^4, the eigenvector residuals under
the oracle's gather stencil on a non-cubic lattice, the spectral sign against the
Schur sign, and the abelian degeneracy.
"""
from __future__ import annotations

import numpy as np

from .wilson import Geometry, gamma5, gamma_matrices, kappa_of_mass


def momenta(dims, antiperiodic_t: bool = True) -> np.ndarray:
    """(V, 4) lattice momenta in the site order: 2 pi n / N, and pi (2n + 1)/N_t in time."""
    geo = Geometry(dims, antiperiodic_t=False)
    n = geo.coords.T.astype(np.float64)
    p = 2.0 * np.pi * n / np.asarray(dims, dtype=np.float64)
    if antiperiodic_t:
        p[:, 3] += np.pi / dims[3]
    return p


def symbols(dims, mass: float, mu: float, C: np.ndarray, antiperiodic_t: bool = True) -> np.ndarray:
    """(V, 12, 12): M(p) for every momentum, index order (spin, colour)."""
    kap = kappa_of_mass(mass)
    gam = gamma_matrices()
    g5 = gamma5()
    p = momenta(dims, antiperiodic_t)
    one = np.eye(4)
    M = np.broadcast_to(np.eye(12, dtype=np.complex128), (p.shape[0], 12, 12)).copy()
    for nu in range(4):
        ef = np.exp(mu) if nu == 3 else 1.0
        eb = np.exp(-mu) if nu == 3 else 1.0
        fwd = np.kron(one + gam[nu], C[nu])
        bwd = np.kron(one - gam[nu], C[nu].conj().T)
        M -= kap * (ef * np.exp(1j * p[:, nu])[:, None, None] * fwd + eb * np.exp(-1j * p[:, nu])[:, None, None] * bwd)
    return np.kron(g5, np.eye(3))[None] @ M


def spectrum(dims, mass: float, mu: float, C: np.ndarray, antiperiodic_t: bool = True):
    """All 12 V eigenvalues (V, 12) with right and left vectors (V, 12, 12) (column k of
    each), w_k^H u_j = delta_kj."""
    lam, Ur = np.linalg.eig(symbols(dims, mass, mu, C, antiperiodic_t))
    Wl = np.conj(np.swapaxes(np.linalg.inv(Ur), -1, -2))
    return lam, Ur, Wl


def eigenvectors(dims, g: np.ndarray, labels, Ur, Wl, antiperiodic_t: bool = True):
    """Right and left eigenvectors (len(labels), V, 4, 3) for (momentum, branch) labels."""
    geo = Geometry(dims, antiperiodic_t=False)
    p = momenta(dims, antiperiodic_t)
    V = geo.volume
    out_r = np.empty((len(labels), V, 4, 3), dtype=np.complex128)
    out_l = np.empty_like(out_r)
    for i, (q, k) in enumerate(labels):
        wave = np.exp(1j * (p[q] @ geo.coords)) / np.sqrt(V)
        u = Ur[q, :, k].reshape(4, 3)
        w = Wl[q, :, k].reshape(4, 3)
        out_r[i] = wave[:, None, None] * np.einsum("vab,sb->vsa", g, u)
        out_l[i] = wave[:, None, None] * np.einsum("vab,sb->vsa", g, w)
    return out_r, out_l


def lowest_eigenpairs(dims, mass: float, mu: float, C: np.ndarray, g: np.ndarray, l: int,
                      antiperiodic_t: bool = True):
    """The l eigenpairs of smallest |lambda| of H on the field g C g^dag: dict with
    lam (l,), R and L (l, V, 4, 3) with L_i^H R_j = delta_ij, labels, separation
    (min over all other eigenvalues of |lambda_i - lambda_j|) and edge
    (|lambda_l|, |lambda_{l+1}|)."""
    lam, Ur, Wl = spectrum(dims, mass, mu, C, antiperiodic_t)
    flat = lam.ravel()
    order = np.argsort(np.abs(flat), kind="stable")
    pick = order[:l]
    labels = [tuple(int(a) for a in np.unravel_index(i, lam.shape)) for i in pick]
    sep = np.array([np.partition(np.abs(flat - flat[i]), 1)[1] for i in pick])
    R, L = eigenvectors(dims, g, labels, Ur, Wl, antiperiodic_t)
    return dict(lam=flat[pick], R=R, L=L, labels=labels, separation=sep,
                edge=(float(np.abs(flat[order[l - 1]])), float(np.abs(flat[order[l]]))))


def tracked_eigenpairs(dims, mass: float, mu: float, C: np.ndarray, g: np.ndarray, labels, lam_ref,
                       antiperiodic_t: bool = True):
    """Eigenpairs of the field g C g^dag that continue given ones: for each (momentum,
    branch) label the eigenvalue of M(p) nearest to lam_ref[i] (C moved by a small
    amount from where the labels were taken).  Returns (lam, R, L, jump) with jump the
    largest distance to the reference, and refuses a pick that is not unique."""
    qs = sorted({q for q, _ in labels})
    M = symbols(dims, mass, mu, C, antiperiodic_t)[qs]
    lam_q, U_q = np.linalg.eig(M)
    W_q = np.conj(np.swapaxes(np.linalg.inv(U_q), -1, -2))
    lam = np.empty(len(labels), dtype=np.complex128)
    new_labels = []
    Ur = np.zeros((max(qs) + 1, 12, 12), dtype=np.complex128)
    Wl = np.zeros_like(Ur)
    for j, q in enumerate(qs):
        Ur[q], Wl[q] = U_q[j], W_q[j]
    for i, (q, _) in enumerate(labels):
        d = np.abs(lam_q[qs.index(q)] - lam_ref[i])
        k = int(np.argmin(d))
        if np.partition(d, 1)[1] <= 2.0 * d[k]:
            raise RuntimeError("eigenvalue tracking is ambiguous")
        lam[i] = lam_q[qs.index(q)][k]
        new_labels.append((q, k))
    R, L = eigenvectors(dims, g, new_labels, Ur, Wl, antiperiodic_t)
    return lam, R, L, float(np.max(np.abs(lam - np.asarray(lam_ref))))


def exact_sign(dims, mass: float, mu: float, C: np.ndarray, g: np.ndarray, psi: np.ndarray,
               antiperiodic_t: bool = True) -> np.ndarray:
    """sgn(H) psi from the full spectral decomposition (eq. spectral_form, every
    eigenvalue's sign): undo g, expand in the plane waves of ``momenta`` (a 4-d FFT
    over (t, z, y, x) after the half-integer temporal phase), apply
    sum_k sgn(Re lambda_k) u_k w_k^H per momentum and transform back."""
    nx, ny, nz, nt = dims
    V = nx * ny * nz * nt
    geo = Geometry(dims, antiperiodic_t=False)
    lam, Ur, Wl = spectrum(dims, mass, mu, C, antiperiodic_t)
    S = np.einsum("qik,qk,qjk->qij", Ur, np.sign(lam.real), Wl.conj())
    shift = np.exp(-1j * np.pi * geo.coords[3] / nt) if antiperiodic_t else np.ones(V)
    phi = np.einsum("vba,vsb->vsa", g.conj(), psi).reshape(V, 12) * shift[:, None]     # g^dag psi
    box = (nt, nz, ny, nx)
    chi = np.fft.fftn(phi.reshape(box + (12,)), axes=(0, 1, 2, 3), norm="ortho").reshape(V, 12)
    chi = np.einsum("qij,qj->qi", S, chi)
    back = np.fft.ifftn(chi.reshape(box + (12,)), axes=(0, 1, 2, 3), norm="ortho").reshape(V, 12)
    back = (back * shift.conj()[:, None]).reshape(V, 4, 3)
    return np.einsum("vab,vsb->vsa", g, back)
