"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the method (no Dirac operator, no Krylov
recursion, no sign function, no derivative).  It only draws random numbers and
shapes them into the canonical host layouts that both sides consume.
"""
from .fields import (  # noqa: F401
    CONFIGS,
    Workload,
    config_rng,
    gauge_transform,
    lattice_volume,
    random_su3,
    random_links,
    uneven_krylov_sizes,
    workload,
    z2_complex_source,
)
