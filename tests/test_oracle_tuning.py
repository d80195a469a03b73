"""Pins of oracle.tuning: the tuning run that picks the Krylov sizes (Sec. 4.1).

* the selection on hand-made (error, time) tables: the fastest candidate within
  the target, skipping faster ones above it, the first of equal times, none;
* the trial vector is (1, ..., 1);
* the error estimate of the full Krylov space (re-biorthogonalised) vanishes, and
  a nested step with inner size >= outer size gives the plain step's error;
* a tuning run on a tiny lattice with times growing in k keeps the smallest
  candidate that meets the target, whose cross-check errors on random vectors are
  of the trial error's order (the paper's observation, checked within 100x).
"""
import numpy as np
import pytest

from oracle import deflation as DF
from oracle import tuning as TU
from oracle.wilson import WilsonOperator, dense_h
from synthetic import random_links, z2_complex_source


def test_selection_tables():
    assert TU.select([1e-3, 1e-9, 1e-10], [1.0, 2.0, 3.0], 1e-8) == 1
    assert TU.select([1e-9, 1e-10], [5.0, 2.0], 1e-8) == 1           # the faster of two that pass
    assert TU.select([1e-12, 1e-3, 1e-9], [3.0, 1.0, 2.0], 1e-8) == 2  # the fastest fails the target
    assert TU.select([1e-9, 1e-9], [2.0, 2.0], 1e-8) == 0             # first of equal times
    assert TU.select([1e-3, 1e-4], [1.0, 2.0], 1e-8) == -1
    assert TU.select([1e-8], [1.0], 1e-8) == 0                         # the target itself passes


def test_trial_vector():
    phi = TU.trial_vector(5)
    assert phi.shape == (5, 4, 3) and np.all(phi == 1.0)


@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 4)
    U = random_links(dims, 0.5, np.random.default_rng(12))
    return dims, U, WilsonOperator(dims, -2.0, 0.3)


def test_full_space_and_nested_limits(tiny):
    dims, U, op = tiny
    phi = TU.trial_vector(op.volume)
    n = 12 * op.volume
    assert TU.sign_error(op, U, phi, n, reorth=True) < 1e-10
    H = dense_h(U, dims, -2.0, 0.3)
    lam, R, L = DF.eigenpairs(H, n)
    assert TU.sign_error(op, U, phi, 1, defl=(lam, R, L)) < 1e-12   # deflating everything is exact
    for k in (12, 24):
        plain = TU.sign_error(op, U, phi, k)
        assert abs(TU.sign_error(op, U, phi, k, k_inner=k) - plain) < 1e-8 * plain   # rounding through (T^2)^-1


def test_tuning_run_on_tiny_lattice(tiny):
    dims, U, op = tiny
    phi = TU.trial_vector(op.volume)
    ks = [8, 16, 32, 64, 96]
    cands = [(k, 0) for k in ks]
    errs_all = [TU.sign_error(op, U, phi, k) for k in ks]
    eps0 = 10.0 * errs_all[3]             # the k = 64 trial error passes 0.1 eps0, k = 32's must not
    assert errs_all[2] > errs_all[3]
    chosen, errs = TU.tuning_run(lambda c: TU.sign_error(op, U, phi, c[0], c[1]), cands, [float(k) for k in ks],
                                 eps0)
    assert errs == errs_all
    want = min(i for i, e in enumerate(errs_all) if e <= 0.1 * eps0)
    assert chosen == want
    r = np.random.default_rng(3)
    vecs = [z2_complex_source(op.volume, r) for _ in range(4)]
    cross, ok = TU.cross_check(lambda v: TU.sign_error(op, U, v, ks[chosen]), vecs, eps0)
    assert max(cross) < 100 * errs[chosen] and min(cross) > errs[chosen] / 100
