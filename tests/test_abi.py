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
    assert lib.tslov_sign_grad(None, None, None, 8, None, 0, None, None, None, None) == ERR_ARG
    assert lib.tslov_kernel_bytes(None, 0) == 0.0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1604_08057_amd import tslov
    with pytest.raises(tslov.TslovLibraryMissing):
        tslov.load_library(str(tmp_path / "libtslov.so"))
