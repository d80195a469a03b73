"""Oracle of the tuning run that picks the Krylov sizes (Sec. 4.1, numerical setup and tuning).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes the Krylov sizes per gauge configuration before production:
a target precision epsilon_0 is chosen, every candidate parameter set
p_i = (k^O_i, k^I_i) (outer size, inner size of the nested step) is run on one
trial vector, its error estimate epsilon_i (eq. error_est, or eq. bA_error_est for
the derivative) and its run time t_i are recorded, candidates with
epsilon_i > epsilon_0 are dropped, and the fastest remaining one is kept.  A
cross-check then evaluates the error of the kept parameters on l random vectors
(l = 20 ... 30 in the paper) and compares the largest with epsilon_0; as a rule of
thumb the trial run aims at a tenth of epsilon_0.  The trial vector is
phi = (1, ..., 1) for the sign function and the sparse (0, phi) for the block
matrix of the derivative.

Readings: the trial target is trial_factor * epsilon_0 (the paper's rule of thumb,
trial_factor = 0.1) and the cross-check passes when every random vector's error is
at most epsilon_0; k^I = 0 denotes the plain projected-matrix step (no nesting).
The selection is a pure function of the (epsilon_i, t_i) table; the errors come
from oracle.deflation.error_estimate over the plain (oracle.tsl) or nested
(oracle.nested) sign, deflated or not, and from oracle.blockderiv.eps_block.
"""
from __future__ import annotations

import numpy as np

from . import blockderiv as BD
from . import deflation as DF
from .nested import nested_matrix_function
from .tsl import tsl_wilson


def trial_vector(volume: int) -> np.ndarray:
    """phi = (1, ..., 1) in the canonical (V, 4, 3) layout."""
    return np.ones((volume, 4, 3), dtype=np.complex128)


def select(eps, times, target: float) -> int:
    """Index of the fastest candidate with eps_i <= target (the first of equal times),
    or -1 if none meets the target."""
    best = -1
    for i, (e, t) in enumerate(zip(eps, times)):
        if e <= target and (best < 0 or t < times[best]):
            best = i
    return best


def sign_error(op, U: np.ndarray, psi: np.ndarray, k_outer: int, k_inner: int = 0, defl=None, **kw) -> float:
    """epsilon_A of eq. error_est for the (deflated) plain or nested TSL sign (keyword
    arguments go to oracle.tsl.tsl)."""
    import torch
    if k_inner:
        kw = dict(kw, f=nested_matrix_function(k_inner))
    if defl is not None:
        lam, R, L = defl
        fn = lambda x: DF.deflated_sign(op, U, x, k_outer, lam, R, L, **kw)  # noqa: E731
    else:
        Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128))

        def fn(x):
            with torch.no_grad():
                return tsl_wilson(op, Ut, torch.from_numpy(np.ascontiguousarray(x)), k_outer, **kw).y.numpy()
    return DF.error_estimate(fn, psi)


def block_error(op, U: np.ndarray, psi: np.ndarray, k_outer: int, nu: int, site: int, X: np.ndarray) -> float:
    """epsilon_B of eq. bA_error_est for the link direction (nu, site, X), source (0, psi)."""
    return BD.eps_block(op, U, psi, k_outer, nu, site, X)


def tuning_run(error_of, candidates, times, eps0: float, trial_factor: float = 0.1):
    """The tuning run on given candidate times: (chosen index, errors) with
    errors[i] = error_of(candidate i) on the trial vector and the trial target
    trial_factor * eps0."""
    errs = [float(error_of(c)) for c in candidates]
    return select(errs, times, trial_factor * eps0), errs


def cross_check(error_of_vector, vectors, eps0: float):
    """(errors of the random vectors, all within eps0)."""
    errs = [float(error_of_vector(v)) for v in vectors]
    return errs, bool(max(errs) <= eps0)
