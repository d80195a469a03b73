"""The C-ABI library loads and exports every function include/tslov.h declares;
host-side argument checks work without a GPU (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tslov.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tslov_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1604_08057_amd import tslov
    if not os.path.exists(tslov.LIB_PATH):
        from paper_1604_08057_amd.build import build
        build()
    return tslov.load_library()


def test_header_declares_the_api():
    names = _declared()
    for n in ("tslov_create", "tslov_destroy", "tslov_set_links", "tslov_apply_dw", "tslov_apply_h",
              "tslov_sign", "tslov_overlap", "tslov_sign_grad", "tslov_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1604_08057_amd import tslov
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(tslov.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", tslov.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_host_side_argument_errors(lib):
    from paper_1604_08057_amd.tslov import ERR_ARG, LatticeDesc
    h = ctypes.c_void_p()
    bad = LatticeDesc((ctypes.c_int * 4)(4, 1, 4, 4), -2.0, 0.3, 1, 0)
    assert lib.tslov_create(ctypes.byref(bad), None, ctypes.byref(h)) == ERR_ARG
    assert b">= 2" in lib.tslov_last_error()
    bad_prec = LatticeDesc((ctypes.c_int * 4)(4, 4, 4, 4), -2.0, 0.3, 1, 7)
    assert lib.tslov_create(ctypes.byref(bad_prec), None, ctypes.byref(h)) == ERR_ARG
    bad_mass = LatticeDesc((ctypes.c_int * 4)(4, 4, 4, 4), -4.0, 0.3, 1, 0)
    assert lib.tslov_create(ctypes.byref(bad_mass), None, ctypes.byref(h)) == ERR_ARG
    assert lib.tslov_create(None, None, ctypes.byref(h)) == ERR_ARG
    assert lib.tslov_sign(None, None, None, 8, None, None) == ERR_ARG
    assert lib.tslov_sign_grad(None, None, None, 8, None, 0, None, None, None, None, None) == ERR_ARG
    assert lib.tslov_overlap_grad(None, None, None, 8, None, 0, None, None, None, None, None) == ERR_ARG
    assert lib.tslov_set_diagnostics(None, 1) == ERR_ARG
    assert lib.tslov_tridiag_sign(None, 4, None, None, None, None, None) == ERR_ARG
    assert lib.tslov_tune_k(None, 1, None, None, 0.0, None, None, 0, None, None, None, None, None) == ERR_ARG
    assert lib.tslov_overlap_solve(None, None, None, 8, 0, 1e-10, 10, None, None) == ERR_ARG
    assert lib.tslov_physical_current(None, 1, None, 8, 1e-10, 10, None, None, None, None, None) == ERR_ARG
    assert lib.tslov_kernel_bytes(None, 0) == 0.0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1604_08057_amd import tslov
    with pytest.raises(tslov.TslovLibraryMissing):
        tslov.load_library(str(tmp_path / "libtslov.so"))


def _tridiag(T):
    import numpy as np
    return np.diag(T).copy(), np.diag(T, -1).real.copy(), np.diag(T, 1).copy()


def test_ritz_values_match_a_dense_eigensolver(lib):
    """The host eigenvalue solver of T_k (Ehrlich-Aberth on the tridiagonal
    recurrence) against LAPACK on the dense matrix: random complex tridiagonal
    matrices up to k = 600 and the oracle's own Lanczos matrix of the 4^4
    workload (k = 64).  Host code only: no device is touched."""
    import numpy as np
    from paper_1604_08057_amd.tslov import ritz_values
    rng = np.random.default_rng(5)
    mats = []
    for k in (1, 2, 7, 60, 600):
        T = np.diag(rng.standard_normal(k) + 1j * rng.standard_normal(k))
        if k > 1:
            T += np.diag(rng.random(k - 1) + 0.1, -1) + np.diag(rng.standard_normal(k - 1) + 1j * rng.standard_normal(k - 1), 1)
        mats.append(T)
    from oracle import grad as GR
    from oracle.wilson import WilsonOperator
    from synthetic import workload
    wl = workload(1)
    mats.append(GR.forward(WilsonOperator(wl.dims, wl.mass, wl.mu), wl.links(), wl.psi(), wl.k)["T"])
    for T in mats:
        ev, sweeps = ritz_values(*_tridiag(T))
        ref = np.linalg.eigvals(T)
        d = np.abs(ev[:, None] - ref[None, :])
        err = max(d.min(axis=1).max(), d.min(axis=0).max()) / np.abs(ref).max()
        assert sweeps >= 0 and err < 1e-12, (T.shape, err, sweeps)
        assert abs(np.abs(ev.real).min() - np.abs(ref.real).min()) < 1e-12 * np.abs(ref).max()


def test_ritz_values_on_the_imaginary_axis(lib):
    """A constructed T whose eigenvalues include +-i (and so one on Re z = 0):
    T = [[0, 1], [-1, 0]] scaled into a larger matrix with separate real block."""
    import numpy as np
    from paper_1604_08057_amd.tslov import ritz_values
    T = np.zeros((4, 4), dtype=np.complex128)
    T[0, 0], T[1, 1] = 0.0, 0.0
    T[1, 0], T[0, 1] = 1.0, -1.0          # eigenvalues +-i
    T[2, 2], T[3, 3] = 2.0, -3.0
    T[2, 1], T[1, 2] = 0.0, 0.0          # decoupled
    T[3, 2], T[2, 3] = 0.5, 0.5
    ev, _ = ritz_values(*_tridiag(T))
    assert np.abs(ev.real).min() < 1e-14
    assert np.allclose(np.sort_complex(ev), np.sort_complex(np.linalg.eigvals(T)), atol=1e-13)
