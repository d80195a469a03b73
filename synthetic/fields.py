"""Seeded synthetic lattice fields in the canonical host layouts.

Canonical layouts (shared contract of the C ABI, the oracle and the tests):

* site index  ``s = x + Nx*(y + Ny*(z + Nz*t))`` with ``dims = (Nx, Ny, Nz, Nt)``;
* gauge links ``U[mu][s][a][b]`` complex128, shape ``(4, V, 3, 3)``, direction
  order x, y, z, t; ``U[mu][s]`` is the link leaving site ``s`` in direction mu;
* spinors ``psi[s][spin][colour]`` complex128, shape ``(V, 4, 3)``.

Streams of ``numpy.random.default_rng([1604, 8057, config, stream])``:
0 links, 1 source psi, 2 probe eta, 3 Krylov-size draws, 4 finite-difference
picks, 5 gauge transformations for tests.

The paper measures on quenched SU(3) ensembles (Sec. 4.1) that are not
available here; random links ``U = exp(i * spread * sum_a c_a lambda_a)`` with
``c_a ~ N(0, 1)`` stand in for them, on the paper's lattice shapes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Gell-Mann basis of su(3), normalised tr(l_a l_b) = 2 delta_ab.  Used only to
# draw random group elements; the method itself never sees it.
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1], _GM[1][1, 0] = -1j, 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2], _GM[4][2, 0] = -1j, 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2], _GM[6][2, 1] = -1j, 1j
_GM[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def config_rng(config: int, stream: int) -> np.random.Generator:
    """Generator for one (workload, stream) pair of the seed scheme above."""
    return np.random.default_rng([1604, 8057, int(config), int(stream)])


def lattice_volume(dims) -> int:
    nx, ny, nz, nt = (int(d) for d in dims)
    return nx * ny * nz * nt


def random_su3(count: int, spread: float, rng: np.random.Generator) -> np.ndarray:
    """``count`` SU(3) matrices ``exp(i*spread*sum_a c_a lambda_a)``, c_a ~ N(0,1).

    The exponential goes through the eigen-decomposition of the Hermitian
    generator, so the result is unitary with unit determinant to rounding.
    """
    c = rng.standard_normal((count, 8))
    herm = spread * np.einsum("na,aij->nij", c, _GM)
    w, q = np.linalg.eigh(herm)
    return np.einsum("nij,nj,nkj->nik", q, np.exp(1j * w), q.conj())


def random_links(dims, spread: float, rng: np.random.Generator) -> np.ndarray:
    """Gauge field of shape ``(4, V, 3, 3)`` drawn as one ``(4, V, 8)`` array."""
    v = lattice_volume(dims)
    return random_su3(4 * v, spread, rng).reshape(4, v, 3, 3)


def forward_neighbours(dims) -> np.ndarray:
    """(4, V) index of the site x + nu for every site x (periodic wrap)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = [x.ravel(), y.ravel(), z.ravel(), t.ravel()]
    n = (nx, ny, nz, nt)
    out = []
    for nu in range(4):
        d = list(c)
        d[nu] = (d[nu] + 1) % n[nu]
        out.append(d[0] + nx * (d[1] + ny * (d[2] + nz * d[3])))
    return np.stack(out)


def links_from_constant(C: np.ndarray, g: np.ndarray, dims) -> np.ndarray:
    """U_nu(x) = g(x) C_nu g(x + nu)^dag for constant C (4, 3, 3) and g (V, 3, 3)."""
    fwd = forward_neighbours(dims)
    return np.stack([np.einsum("vab,bc,vdc->vad", g, C[nu], g[fwd[nu]].conj()) for nu in range(4)])


def rotated_constant_links(dims, spread: float, rng: np.random.Generator):
    """(U, C, g): a constant SU(3) link per direction, C of shape (4, 3, 3) drawn like
    ``random_su3`` with ``spread``, seen through a random SU(3) gauge rotation g(x)
    (shape (V, 3, 3)): U_nu(x) = g(x) C_nu g(x + nu)^dag.  Link by link the field
    looks random; its spectrum is that of the translation-invariant field C."""
    v = lattice_volume(dims)
    C = random_su3(4, spread, rng)
    g = random_su3(v, 1.0, rng)
    return links_from_constant(C, g, dims), C, g


def z2_complex_source(volume: int, rng: np.random.Generator, count: int | None = None) -> np.ndarray:
    """Components ``(s1 + i*s2)/sqrt(2)`` with s1, s2 = +-1 i.i.d.; shape ``(V, 4, 3)``."""
    shape = (volume, 4, 3) if count is None else (count, volume, 4, 3)
    s = rng.integers(0, 2, size=shape + (2,)) * 2 - 1
    return (s[..., 0] + 1j * s[..., 1]) / np.sqrt(2.0)


def gauge_transform(volume: int, rng: np.random.Generator, spread: float = 1.0) -> np.ndarray:
    """Random SU(3) matrix per site, shape ``(V, 3, 3)`` (gauge-covariance tests)."""
    return random_su3(volume, spread, rng)


def uneven_krylov_sizes(count: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    """Per-source Krylov sizes drawn uniformly from the integers ``[lo, hi]``."""
    return rng.integers(lo, hi + 1, size=count)


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, operator parameters and Krylov size."""

    config: int
    name: str
    dims: tuple
    spread: float
    mass: float
    mu: float
    k: int
    sources: int = 1
    k_range: tuple | None = None
    n_deflate: int = 0
    precision: str = "fp64"
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        return lattice_volume(self.dims)

    def links(self) -> np.ndarray:
        if self.extra.get("field") == "rotated-constant":
            return self.constant_field()[0]
        return random_links(self.dims, self.spread, config_rng(self.config, 0))

    def constant_field(self):
        """(U, C, g) of a rotated-constant workload (see ``rotated_constant_links``);
        the draw index picks one seeded field of that family."""
        rng = np.random.default_rng([1604, 8057, self.config, 0, int(self.extra["draw"])])
        return rotated_constant_links(self.dims, self.spread, rng)

    def psi(self) -> np.ndarray:
        if self.sources == 1:
            return z2_complex_source(self.volume, config_rng(self.config, 1))
        return z2_complex_source(self.volume, config_rng(self.config, 1), self.sources)

    def eta(self) -> np.ndarray:
        if self.sources == 1:
            return z2_complex_source(self.volume, config_rng(self.config, 2))
        return z2_complex_source(self.volume, config_rng(self.config, 2), self.sources)

    def krylov_sizes(self) -> np.ndarray:
        if self.k_range is None:
            return np.full(self.sources, self.k)
        return uneven_krylov_sizes(self.sources, self.k_range[0], self.k_range[1],
                                   config_rng(self.config, 3))


# The five workloads: (Nx, Ny, Nz, Nt).  "N x M^3" means Nt = N, spatial M^3.
CONFIGS = {
    1: Workload(1, "tiny 4^4", (4, 4, 4, 4), 0.5, -2.0, 0.3, 64),
    2: Workload(2, "8^4 fp64", (8, 8, 8, 8), 0.4, -2.0, 0.2, 200),
    3: Workload(3, "14x14^3 mixed", (14, 14, 14, 14), 0.35, -2.0, 0.3, 400, precision="mixed"),
    4: Workload(4, "6x18^3 batched", (18, 18, 18, 6), 0.35, -2.0, 0.5, 400, sources=32,
                k_range=(100, 400), precision="mixed"),
    # 16^4: a gauge-rotated constant field, so that the 20 lowest eigenpairs are known
    # exactly; draw 10 of that family keeps them >= 6.4e-3 away from every other
    # eigenvalue and |Re lambda| >= 0.025.
    5: Workload(5, "16^4 deflated", (16, 16, 16, 16), 0.35, -2.0, 0.3, 400, n_deflate=20,
                extra={"field": "rotated-constant", "draw": 10}),
    # 3x4^3 (the size of the paper's check of the current's divergence, mu = 0.3) with
    # smooth links and a mass inside the overlap window: min |Re lambda(H)| = 0.29, so the
    # TSL approximation converges (eps_A 1.4e-13 at k = 240) and D_ov can be inverted
    6: Workload(6, "3x4^3 physical current", (4, 4, 4, 3), 0.1, -1.0, 0.3, 240, sources=4),
}


def workload(config: int) -> Workload:
    return CONFIGS[int(config)]
