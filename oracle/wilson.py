"""Oracle Wilson-Dirac operator at chemical potential mu (App. A, eq. WD_op, WD_G).

    D_w(mu) psi(x) = psi(x) - kappa * sum_nu [ e^{+mu d_{nu,t}} (1 + g_nu) U_nu(x) psi(x + nu)
                                             + e^{-mu d_{nu,t}} (1 - g_nu) U_nu(x - nu)^dag psi(x - nu) ]

Readings of the text (App. A is silent or inconsistent on these):
* kappa = 1/(2 m + 8) with the signed Wilson mass m (m = -2 gives kappa = 1/4);
* U_{-nu}(x) is U_nu(x - nu)^dagger; the projector (1 + g_nu) sits on the forward hop;
* e^{+-mu} multiplies every temporal hop, not only the boundary ones;
* boundary conditions: periodic in x, y, z and antiperiodic in t (a factor -1 on
  every hop that crosses between t = Nt-1 and t = 0);
* Euclidean Dirac matrices in the chiral basis g_k = [[0, -i s_k], [i s_k, 0]],
  g_4 = [[0, 1], [1, 0]], so g_5 = g_1 g_2 g_3 g_4 = diag(1, 1, -1, -1);
* H(mu) = g_5 D_w(mu) (Sec. 1, eq. overlap), and H(mu)^dagger = H(-mu).

Three independent evaluations are provided: a gather stencil in torch (any
lattice, differentiable in U), a dense 12V x 12V builder that loops over links
(tiny lattices), and the free-field closed form for plane waves.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_S = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
      np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
      np.array([[1, 0], [0, -1]], dtype=np.complex128)]
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def gamma_matrices() -> np.ndarray:
    """Euclidean Dirac matrices g_1..g_4 (index 0..3 = x, y, z, t), chiral basis."""
    g = [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _S]
    g.append(np.block([[_Z2, _I2], [_I2, _Z2]]))
    return np.stack(g)


def gamma5() -> np.ndarray:
    g = gamma_matrices()
    return g[0] @ g[1] @ g[2] @ g[3]


def kappa_of_mass(mass: float) -> float:
    """Hopping parameter kappa = 1/(2 m + 8) (App. A), m the signed Wilson mass."""
    return 1.0 / (2.0 * mass + 8.0)


class Geometry:
    """Site numbering s = x + Nx*(y + Ny*(z + Nz*t)) and hop tables with boundary signs."""

    def __init__(self, dims, antiperiodic_t: bool = True):
        self.dims = tuple(int(d) for d in dims)
        nx, ny, nz, nt = self.dims
        self.volume = nx * ny * nz * nt
        t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                                 indexing="ij")
        coords = np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()])  # (4, V), site order
        self.coords = coords
        self.fwd = np.empty((4, self.volume), dtype=np.int64)
        self.bwd = np.empty((4, self.volume), dtype=np.int64)
        self.sign_fwd = np.ones((4, self.volume))
        self.sign_bwd = np.ones((4, self.volume))
        for nu in range(4):
            up = coords.copy()
            up[nu] = (up[nu] + 1) % self.dims[nu]
            dn = coords.copy()
            dn[nu] = (dn[nu] - 1) % self.dims[nu]
            self.fwd[nu] = self.index(up)
            self.bwd[nu] = self.index(dn)
        if antiperiodic_t:
            self.sign_fwd[3, coords[3] == nt - 1] = -1.0
            self.sign_bwd[3, coords[3] == 0] = -1.0

    def index(self, c) -> np.ndarray:
        nx, ny, nz, _ = self.dims
        return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))


class WilsonOperator:
    """Gather stencil for D_w(mu) and H(mu) on complex128 torch tensors (CPU).

    ``U`` has shape (4, V, 3, 3); spinors have shape (V, 4, 3).  Every call is
    differentiable in both U and the spinor, so torch autograd can take the
    all-links derivative of anything built from it.
    """

    def __init__(self, dims, mass: float, mu: float, antiperiodic_t: bool = True):
        self.geom = Geometry(dims, antiperiodic_t)
        self.kappa = kappa_of_mass(mass)
        self.mu = float(mu)
        self.gam = torch.from_numpy(gamma_matrices())
        self.g5 = torch.from_numpy(np.diag(gamma5()).copy())
        self.fwd = torch.from_numpy(self.geom.fwd)
        self.bwd = torch.from_numpy(self.geom.bwd)
        self.sf = torch.from_numpy(self.geom.sign_fwd).to(torch.complex128)
        self.sb = torch.from_numpy(self.geom.sign_bwd).to(torch.complex128)

    @property
    def volume(self) -> int:
        return self.geom.volume

    def hop(self, U: torch.Tensor, psi: torch.Tensor, mu: float) -> torch.Tensor:
        """sum_nu [e^{mu d} (1+g) U(x) psi(x+nu) + e^{-mu d} (1-g) U(x-nu)^dag psi(x-nu)]."""
        out = torch.zeros_like(psi)
        for nu in range(4):
            ef = math.exp(mu) if nu == 3 else 1.0
            eb = math.exp(-mu) if nu == 3 else 1.0
            g = self.gam[nu]
            up = torch.einsum("vab,vsb->vsa", U[nu], psi[self.fwd[nu]])
            up = up + torch.einsum("st,vta->vsa", g, up)
            out = out + (ef * self.sf[nu])[:, None, None] * up
            ub = U[nu][self.bwd[nu]]
            dn = torch.einsum("vba,vsb->vsa", ub.conj(), psi[self.bwd[nu]])
            dn = dn - torch.einsum("st,vta->vsa", g, dn)
            out = out + (eb * self.sb[nu])[:, None, None] * dn
        return out

    def dw(self, U, psi, mu=None):
        """D_w(mu) psi (eq. WD_op)."""
        mu = self.mu if mu is None else mu
        return psi - self.kappa * self.hop(U, psi, mu)

    def dw_dag(self, U, psi, mu=None):
        """D_w(mu)^dagger psi = g5 D_w(-mu) g5 psi."""
        mu = self.mu if mu is None else mu
        return self.g5[None, :, None] * self.dw(U, self.g5[None, :, None] * psi, -mu)

    def h(self, U, psi, mu=None):
        """H(mu) psi = g5 D_w(mu) psi."""
        return self.g5[None, :, None] * self.dw(U, psi, mu)

    def h_dag(self, U, psi, mu=None):
        """H(mu)^dagger psi = H(-mu) psi."""
        mu = self.mu if mu is None else mu
        return self.h(U, psi, -mu)


def dense_dw(U: np.ndarray, dims, mass: float, mu: float, antiperiodic_t: bool = True) -> np.ndarray:
    """Dense D_w(mu) as a (12V, 12V) matrix, index 12*s + 3*spin + colour.

    Written independently of the stencil: it walks over the links U_nu(x) and
    places each link's two hopping blocks (x -> x+nu and x+nu -> x) directly.
    Intended for V <= 256.
    """
    nx, ny, nz, nt = dims
    vol = nx * ny * nz * nt
    kap = kappa_of_mass(mass)
    gam = gamma_matrices()
    one = np.eye(4)
    D = np.zeros((vol, 4, 3, vol, 4, 3), dtype=np.complex128)
    for s in range(vol):
        D[s, :, :, s, :, :] = np.einsum("st,ab->satb", one, np.eye(3))
    ext = (nx, ny, nz, nt)
    for s in range(vol):
        c = [s % nx, (s // nx) % ny, (s // (nx * ny)) % nz, s // (nx * ny * nz)]
        for nu in range(4):
            c2 = list(c)
            c2[nu] += 1
            wrap = c2[nu] == ext[nu]
            c2[nu] %= ext[nu]
            s2 = c2[0] + nx * (c2[1] + ny * (c2[2] + nz * c2[3]))
            bc = -1.0 if (nu == 3 and wrap and antiperiodic_t) else 1.0
            e = math.exp(mu) if nu == 3 else 1.0
            link = U[nu, s]
            # forward hop at s picks psi(s2) through U_nu(s)
            D[s, :, :, s2, :, :] += -kap * e * bc * np.einsum("st,ab->satb", one + gam[nu], link)
            # backward hop at s2 picks psi(s) through U_nu(s)^dagger
            D[s2, :, :, s, :, :] += -kap * bc / e * np.einsum("st,ab->satb", one - gam[nu],
                                                             link.conj().T)
    return D.reshape(12 * vol, 12 * vol)


def dense_h(U, dims, mass, mu, antiperiodic_t=True) -> np.ndarray:
    """Dense H(mu) = g5 D_w(mu)."""
    vol = int(np.prod(dims))
    g5 = np.kron(np.eye(vol), np.kron(gamma5(), np.eye(3)))
    return g5 @ dense_dw(U, dims, mass, mu, antiperiodic_t)


def free_field_symbol(p, mass: float, mu: float) -> np.ndarray:
    """4x4 spin matrix of D_w(mu) on a plane wave e^{i p.x} chi with U = 1.

    With p4 -> p4 - i mu the temporal factor e^{+-mu} e^{+-i p4} becomes
    e^{+-i (p4 - i mu)}, and each direction contributes
    -kappa [(1+g) e^{i p} + (1-g) e^{-i p}] = -2 kappa [cos p + i g sin p].
    Antiperiodic time means p4 = pi (2n + 1)/Nt.
    """
    kap = kappa_of_mass(mass)
    gam = gamma_matrices()
    pt = np.array(p, dtype=np.complex128)
    pt[3] = pt[3] - 1j * mu
    d = np.eye(4, dtype=np.complex128)
    for nu in range(4):
        d = d - 2 * kap * (np.cos(pt[nu]) * np.eye(4) + 1j * np.sin(pt[nu]) * gam[nu])
    return d


def plane_wave(dims, p, chi: np.ndarray) -> np.ndarray:
    """Spinor field e^{i p.x} chi[spin, colour] in the canonical (V, 4, 3) layout."""
    g = Geometry(dims, antiperiodic_t=False)
    phase = np.exp(1j * (np.asarray(p, dtype=float) @ g.coords))
    return phase[:, None, None] * chi[None, :, :]
