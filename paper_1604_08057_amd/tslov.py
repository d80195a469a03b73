"""Thin Python binding of the tslov C ABI (``include/tslov.h``).

Argument marshalling only: every step of the computation runs in the HIP
library ``libtslov.so``.  Tensors are torch CUDA (HIP) tensors in the canonical
layouts: links complex128 ``(4, V, 3, 3)``, spinors complex128 ``(V, 4, 3)``
with site index ``x + Nx*(y + Ny*(z + Nz*t))``.  PyTorch provides device
memory and the stream; nothing here computes.

Importing this module does not load the library; the first use does, and
raises ``TslovLibraryMissing`` if it has not been built
(``python -m paper_1604_08057_amd.build``).  There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtslov.so")

OK, ERR_ARG, ERR_HIP, ERR_OOM, ERR_BREAKDOWN, ERR_SIGN_UNDEFINED, ERR_NOT_CONVERGED = range(7)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_HIP", 3: "ERR_OOM", 4: "ERR_BREAKDOWN",
                5: "ERR_SIGN_UNDEFINED", 6: "ERR_NOT_CONVERGED"}
PRECISIONS = {"fp64": 0, "mixed": 1, "fp32links": 2}

# Bits of Info.flags and of tslov_set_diagnostics.
FLAG_SIGN_STAGNATED, FLAG_GRAD_FP32_VECTORS, FLAG_RITZ_UNSETTLED = 1, 2, 4
DIAG_EPS_A = 1

# Kernel classes of tslov_timing_read / tslov_kernel_bytes.
KERNEL_FWD_PAIR, KERNEL_BWD_PAIR, KERNEL_APPLY = 0, 1, 2

EXPORTS = ["tslov_create", "tslov_destroy", "tslov_last_error", "tslov_set_links", "tslov_apply_dw",
           "tslov_apply_h", "tslov_sign", "tslov_overlap", "tslov_sign_grad", "tslov_sign_grad_batched",
           "tslov_current_estimate", "tslov_error_estimate", "tslov_lanczos_matrix", "tslov_dense_sign", "tslov_timing_enable",
           "tslov_timing_read", "tslov_kernel_bytes", "tslov_set_pair_ns", "tslov_get_pair_ns", "tslov_set_graphs", "tslov_set_apply_chunk",
           "tslov_get_apply_chunk", "tslov_overlap_grad", "tslov_tridiag_sign", "tslov_ritz_values",
           "tslov_set_diagnostics", "tslov_apply_h_noalloc", "tslov_set_nested", "tslov_block_sign",
           "tslov_block_error_estimate", "tslov_tune_k", "tslov_overlap_solve", "tslov_physical_current",
           "tslov_set_cg_operator", "tslov_block_sign_deflated", "tslov_block_error_estimate_deflated",
           "tslov_sign_grad_batched_deflated", "tslov_current_estimate_deflated"]


class TslovLibraryMissing(ImportError):
    pass


class TslovError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class LatticeDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("mass", ctypes.c_double), ("mu", ctypes.c_double),
                ("antiperiodic_t", ctypes.c_int), ("precision", ctypes.c_int)]


class InfoStruct(ctypes.Structure):
    _fields_ = [("k_used", ctypes.c_int), ("breakdown", ctypes.c_int), ("newton_iters", ctypes.c_int),
                ("cg_iters", ctypes.c_int), ("flags", ctypes.c_int), ("reserved", ctypes.c_int),
                ("norm_x", ctypes.c_double), ("min_abs_re_ritz", ctypes.c_double), ("norm_T", ctypes.c_double),
                ("biorth_err", ctypes.c_double), ("eps_A", ctypes.c_double), ("ms", ctypes.c_double * 6)]


class LinkDirection(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int), ("site", ctypes.c_int), ("X", ctypes.c_double * 18)]


class DeflationStruct(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int), ("R", ctypes.c_void_p), ("L", ctypes.c_void_p),
                ("lambda_", ctypes.POINTER(ctypes.c_double))]


@dataclass
class Info:
    k_used: int
    breakdown: int
    newton_iters: int
    norm_x: float
    ms: tuple
    cg_iters: int = 0            # shifted-solve iterations of the deflated derivative
    flags: int = 0               # FLAG_* bits
    min_abs_re_ritz: float = float("nan")
    norm_T: float = float("nan")
    biorth_err: float = 0.0
    eps_A: float = float("nan")

    @classmethod
    def of(cls, s: InfoStruct) -> "Info":
        return cls(s.k_used, s.breakdown, s.newton_iters, s.norm_x, tuple(s.ms), s.cg_iters, s.flags,
                   s.min_abs_re_ritz, s.norm_T, s.biorth_err, s.eps_A)


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libtslov.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise TslovLibraryMissing(f"{p} is missing; build it with `python -m paper_1604_08057_amd.build`")
    lib = ctypes.CDLL(p)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "tslov_create": ([ctypes.POINTER(LatticeDesc), vp, ctypes.POINTER(vp)], ci),
        "tslov_destroy": ([vp], None),
        "tslov_last_error": ([], ctypes.c_char_p),
        "tslov_set_links": ([vp, vp], ci),
        "tslov_apply_dw": ([vp, vp, vp, ci], ci),
        "tslov_apply_h": ([vp, vp, vp, ci], ci),
        "tslov_apply_h_noalloc": ([vp, vp, vp, ci], ci),
        "tslov_sign": ([vp, vp, vp, ci, ctypes.POINTER(DeflationStruct), ctypes.POINTER(InfoStruct)], ci),
        "tslov_overlap": ([vp, vp, vp, ci, ctypes.POINTER(DeflationStruct), ctypes.POINTER(InfoStruct)], ci),
        "tslov_sign_grad": ([vp, vp, vp, ci, ctypes.POINTER(DeflationStruct), ci, ctypes.POINTER(cd), vp, vp, vp,
                             ctypes.POINTER(InfoStruct)], ci),
        "tslov_overlap_grad": ([vp, vp, vp, ci, ctypes.POINTER(DeflationStruct), ci, ctypes.POINTER(cd), vp, vp, vp,
                                ctypes.POINTER(InfoStruct)], ci),
        "tslov_sign_grad_batched": ([vp, ci, vp, vp, ctypes.POINTER(ci), ctypes.POINTER(cd), vp, vp, vp,
                                     ctypes.POINTER(InfoStruct)], ci),
        "tslov_tridiag_sign": ([vp, ci, ctypes.POINTER(cd), ctypes.POINTER(cd), ctypes.POINTER(cd), vp,
                                ctypes.POINTER(InfoStruct)], ci),
        "tslov_ritz_values": ([ci, ctypes.POINTER(cd), ctypes.POINTER(cd), ctypes.POINTER(cd), ctypes.POINTER(cd),
                               ctypes.POINTER(ci)], ci),
        "tslov_set_diagnostics": ([vp, ci], ci),
        "tslov_set_nested": ([vp, ci], ci),
        "tslov_block_sign": ([vp, ci, ci, ctypes.POINTER(cd), vp, vp, ci, vp, vp, ctypes.POINTER(InfoStruct)], ci),
        "tslov_block_error_estimate": ([vp, ci, ci, ctypes.POINTER(cd), vp, ci, ctypes.POINTER(cd)], ci),
        "tslov_block_sign_deflated": ([vp, ci, ci, ctypes.POINTER(cd), vp, vp, ci, ctypes.POINTER(DeflationStruct), vp,
                                       vp, ctypes.POINTER(InfoStruct)], ci),
        "tslov_block_error_estimate_deflated": ([vp, ci, ci, ctypes.POINTER(cd), vp, ci,
                                                 ctypes.POINTER(DeflationStruct), ctypes.POINTER(cd)], ci),
        "tslov_overlap_solve": ([vp, vp, vp, ci, ci, cd, ci, ctypes.POINTER(ci), ctypes.POINTER(cd)], ci),
        "tslov_physical_current": ([vp, ci, vp, ci, cd, ci, vp, vp, vp, ctypes.POINTER(ci), ctypes.POINTER(cd)], ci),
        "tslov_tune_k": ([vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci), cd, ctypes.POINTER(DeflationStruct),
                          ctypes.POINTER(LinkDirection), ci, vp, ctypes.POINTER(cd), ctypes.POINTER(cd),
                          ctypes.POINTER(ci), ctypes.POINTER(cd)], ci),
        "tslov_current_estimate": ([vp, ci, vp, ctypes.POINTER(ci), vp, vp, vp, ctypes.POINTER(cd),
                                    ctypes.POINTER(InfoStruct)], ci),
        "tslov_error_estimate": ([vp, vp, ci, ctypes.POINTER(DeflationStruct), ctypes.POINTER(cd)], ci),
        "tslov_lanczos_matrix": ([vp, vp, ci, vp, ctypes.POINTER(InfoStruct)], ci),
        "tslov_dense_sign": ([vp, vp, ci, vp, vp, vp, ctypes.POINTER(ci)], ci),
        "tslov_timing_enable": ([vp, ci], ci),
        "tslov_timing_read": ([vp, ci, ctypes.POINTER(ci), ctypes.POINTER(cd)], ci),
        "tslov_kernel_bytes": ([vp, ci], cd),
        "tslov_set_pair_ns": ([vp, ci], ci),
        "tslov_set_cg_operator": ([vp, ci], ci),
        "tslov_sign_grad_batched_deflated": ([vp, ci, vp, vp, ctypes.POINTER(ci), ctypes.POINTER(DeflationStruct),
                                              ctypes.POINTER(cd), vp, vp, vp, ctypes.POINTER(InfoStruct)], ci),
        "tslov_current_estimate_deflated": ([vp, ci, vp, ctypes.POINTER(ci), ctypes.POINTER(DeflationStruct), vp, vp,
                                             vp, ctypes.POINTER(cd), ctypes.POINTER(InfoStruct)], ci),
        "tslov_set_graphs": ([vp, ci], ci),
        "tslov_set_apply_chunk": ([vp, ci], ci),
        "tslov_get_apply_chunk": ([vp, ctypes.POINTER(ci)], ci),
        "tslov_get_pair_ns": ([vp, ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if path is None:
        _lib = lib
    return lib


def _check(lib, status: int):
    if status != OK:
        raise TslovError(status, lib.tslov_last_error().decode())


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One lattice, operator parameters and workspace on the current HIP device."""

    def __init__(self, dims, mass: float, mu: float, antiperiodic_t: bool = True, precision: str = "fp64",
                 device: int | None = None):
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.volume = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.precision = precision
        d = LatticeDesc((ctypes.c_int * 4)(*self.dims), float(mass), float(mu), int(bool(antiperiodic_t)),
                        PRECISIONS[precision])
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _check(self.lib, self.lib.tslov_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream),
                                                   ctypes.byref(h)))
        self.handle = h
        self._links = None

    # ------------------------------------------------------------------ helpers
    def _spinor(self, x: torch.Tensor, name: str) -> torch.Tensor:
        if x.dtype != torch.complex128 or x.device != self.device or tuple(x.shape) != (self.volume, 4, 3):
            raise ValueError(f"{name} must be a complex128 tensor of shape ({self.volume}, 4, 3) on {self.device}")
        return x.contiguous()

    def _new_spinor(self) -> torch.Tensor:
        return torch.empty((self.volume, 4, 3), dtype=torch.complex128, device=self.device)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.tslov_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ API
    def set_links(self, U: torch.Tensor):
        if U.dtype != torch.complex128 or U.device != self.device or tuple(U.shape) != (4, self.volume, 3, 3):
            raise ValueError(f"links must be complex128 of shape (4, {self.volume}, 3, 3) on {self.device}")
        self._links = U.contiguous()
        _check(self.lib, self.lib.tslov_set_links(self.handle, _ptr(self._links)))

    def apply_dw(self, x: torch.Tensor, dagger: bool = False) -> torch.Tensor:
        x = self._spinor(x, "x")
        out = self._new_spinor()
        _check(self.lib, self.lib.tslov_apply_dw(self.handle, _ptr(x), _ptr(out), int(dagger)))
        return out

    def apply_h(self, x: torch.Tensor, dagger: bool = False) -> torch.Tensor:
        x = self._spinor(x, "x")
        out = self._new_spinor()
        _check(self.lib, self.lib.tslov_apply_h(self.handle, _ptr(x), _ptr(out), int(dagger)))
        return out

    def apply_h_noalloc(self, x: torch.Tensor, out: torch.Tensor, dagger: bool = False) -> torch.Tensor:
        """apply_h with no device allocation in the library (staging in its static
        per-device array); the caller provides out."""
        x = self._spinor(x, "x")
        out = self._spinor(out, "out")
        _check(self.lib, self.lib.tslov_apply_h_noalloc(self.handle, _ptr(x), _ptr(out), int(dagger)))
        return out

    def deflation(self, R: torch.Tensor, L: torch.Tensor, lam) -> "Deflation":
        """Eigenpairs of H for deflation: R, L complex128 (l, V, 4, 3) on the device
        (L_i^H R_j = delta_ij), lam: l complex eigenvalues (host)."""
        return Deflation(self, R, L, lam)

    def sign(self, psi: torch.Tensor, k: int, out: torch.Tensor | None = None, defl: "Deflation | None" = None):
        psi = self._spinor(psi, "psi")
        out = self._new_spinor() if out is None else out
        info = InfoStruct()
        d = None if defl is None else ctypes.byref(defl.struct)
        _check(self.lib, self.lib.tslov_sign(self.handle, _ptr(psi), _ptr(out), int(k), d, ctypes.byref(info)))
        return out, Info.of(info)

    def overlap(self, psi: torch.Tensor, k: int, out: torch.Tensor | None = None, defl: "Deflation | None" = None):
        psi = self._spinor(psi, "psi")
        out = self._new_spinor() if out is None else out
        info = InfoStruct()
        d = None if defl is None else ctypes.byref(defl.struct)
        _check(self.lib, self.lib.tslov_overlap(self.handle, _ptr(psi), _ptr(out), int(k), d, ctypes.byref(info)))
        return out, Info.of(info)

    def error_estimate(self, psi: torch.Tensor, k: int, defl: "Deflation | None" = None) -> float:
        psi = self._spinor(psi, "psi")
        eps = ctypes.c_double()
        d = None if defl is None else ctypes.byref(defl.struct)
        _check(self.lib, self.lib.tslov_error_estimate(self.handle, _ptr(psi), int(k), d, ctypes.byref(eps)))
        return eps.value

    def sign_grad(self, eta: torch.Tensor, psi: torch.Tensor, k: int, want_dpsi: bool = False,
                  dU: torch.Tensor | None = None, defl: "Deflation | None" = None, recompute: int = 0,
                  want_y: bool = False):
        """S = Re <eta|TSL_k(psi)>, dS/dU (and dS/dpsi); recompute = m > 0 holds m + 2
        steps of Krylov vectors and regenerates them in segments of m for the reverse pass.
        With want_y the approximation y = TSL_k(psi) itself is returned too (as a fifth value)."""
        eta = self._spinor(eta, "eta")
        psi = self._spinor(psi, "psi")
        if dU is None:
            dU = torch.empty((4, self.volume, 3, 3), dtype=torch.complex128, device=self.device)
        dpsi = self._new_spinor() if want_dpsi else None
        y = self._new_spinor() if want_y else None
        S = ctypes.c_double()
        info = InfoStruct()
        d = None if defl is None else ctypes.byref(defl.struct)
        _check(self.lib, self.lib.tslov_sign_grad(self.handle, _ptr(eta), _ptr(psi), int(k), d, int(recompute),
                                                  ctypes.byref(S), _ptr(dU), _ptr(dpsi), _ptr(y), ctypes.byref(info)))
        if want_y:
            return S.value, dU, dpsi, Info.of(info), y
        return S.value, dU, dpsi, Info.of(info)

    def overlap_grad(self, eta: torch.Tensor, psi: torch.Tensor, k: int, defl: "Deflation | None" = None,
                     recompute: int = 0):
        """S = Re <eta|D_ov|psi>, dS/dU, dS/dpsi and D_ov psi."""
        eta = self._spinor(eta, "eta")
        psi = self._spinor(psi, "psi")
        dU = torch.empty((4, self.volume, 3, 3), dtype=torch.complex128, device=self.device)
        dpsi = self._new_spinor()
        dov = self._new_spinor()
        S = ctypes.c_double()
        info = InfoStruct()
        d = None if defl is None else ctypes.byref(defl.struct)
        _check(self.lib, self.lib.tslov_overlap_grad(self.handle, _ptr(eta), _ptr(psi), int(k), d, int(recompute),
                                                     ctypes.byref(S), _ptr(dU), _ptr(dpsi), _ptr(dov),
                                                     ctypes.byref(info)))
        return S.value, dU, dpsi, dov, Info.of(info)

    def _sources(self, x: torch.Tensor, name: str) -> torch.Tensor:
        shape = (x.shape[0], self.volume, 4, 3)
        if x.dtype != torch.complex128 or x.device != self.device or tuple(x.shape) != shape:
            raise ValueError(f"{name} must be complex128 of shape (nsrc, {self.volume}, 4, 3) on {self.device}")
        return x.contiguous()

    def sign_grad_batched(self, eta: torch.Tensor, psi: torch.Tensor, ks, want_dpsi: bool = False,
                          want_y: bool = False, defl: "Deflation | None" = None):
        """Per-source S_s, dS_s/dU and (optionally) dS_s/dpsi_s for a batch (nsrc, V, 4, 3);
        with want_y also every y_s = TSL(psi_s) (a fifth value); with defl each source as
        the deflated single-source derivative."""
        psi = self._sources(psi, "psi")
        eta = self._sources(eta, "eta")
        n = psi.shape[0]
        if eta.shape[0] != n or len(ks) != n:
            raise ValueError("eta, psi and ks must have the same number of sources")
        k = (ctypes.c_int * n)(*[int(v) for v in ks])
        S = (ctypes.c_double * n)()
        infos = (InfoStruct * n)()
        dU = torch.empty((n, 4, self.volume, 3, 3), dtype=torch.complex128, device=self.device)
        dpsi = torch.empty_like(psi) if want_dpsi else None
        y = torch.empty_like(psi) if want_y else None
        if defl is None:
            st = self.lib.tslov_sign_grad_batched(self.handle, n, _ptr(eta), _ptr(psi), k, S, _ptr(dU), _ptr(dpsi),
                                                  _ptr(y), infos)
        else:
            st = self.lib.tslov_sign_grad_batched_deflated(self.handle, n, _ptr(eta), _ptr(psi), k,
                                                           ctypes.byref(defl.struct), S, _ptr(dU), _ptr(dpsi),
                                                           _ptr(y), infos)
        _check(self.lib, st)
        if want_y:
            return list(S), dU, dpsi, [Info.of(i) for i in infos], y
        return list(S), dU, dpsi, [Info.of(i) for i in infos]

    def current_estimate(self, xi: torch.Tensor, ks, divergence: bool = True, ward: bool = True,
                         defl: "Deflation | None" = None):
        """j (4, V) = mean over sources of the U(1) link derivatives of Re <g5 xi|sgn(H)|xi>,
        with divergence and total current per site and the per-sample Ward residual;
        with defl the deflated sign (the eigenpairs' motion included)."""
        xi = self._sources(xi, "xi")
        n = xi.shape[0]
        if len(ks) != n:
            raise ValueError("one Krylov size per source")
        k = (ctypes.c_int * n)(*[int(v) for v in ks])
        j = torch.empty((4, self.volume), dtype=torch.float64, device=self.device)
        div = torch.empty(self.volume, dtype=torch.float64, device=self.device) if divergence else None
        tot = torch.empty(self.volume, dtype=torch.float64, device=self.device) if divergence else None
        w = ctypes.c_double()
        infos = (InfoStruct * n)()
        wp = ctypes.byref(w) if ward else None
        if defl is None:
            st = self.lib.tslov_current_estimate(self.handle, n, _ptr(xi), k, _ptr(j), _ptr(div), _ptr(tot), wp, infos)
        else:
            st = self.lib.tslov_current_estimate_deflated(self.handle, n, _ptr(xi), k, ctypes.byref(defl.struct),
                                                          _ptr(j), _ptr(div), _ptr(tot), wp, infos)
        _check(self.lib, st)
        return j, div, tot, (w.value if ward else None), [Info.of(i) for i in infos]

    def lanczos_matrix(self, psi: torch.Tensor, k: int):
        """T_k (k x k complex128 on the host) of the two-sided Lanczos process from psi."""
        import numpy as np
        psi = self._spinor(psi, "psi")
        T = np.zeros((k, k), dtype=np.complex128)
        info = InfoStruct()
        _check(self.lib, self.lib.tslov_lanczos_matrix(self.handle, _ptr(psi), int(k),
                                                       T.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info)))
        return T, Info.of(info)

    def tridiag_sign(self, diag, sub, sup):
        """sgn(T) e_1 for the tridiagonal T (host sequences: k complex diagonal, k-1 real
        sub-diagonal T_{j+1,j}, k-1 complex super-diagonal T_{j,j+1}); returns (c, Info)."""
        a, b, g = _tridiag_arrays(diag, sub, sup)
        k = len(diag)
        c = torch.empty(k, dtype=torch.complex128, device=self.device)
        info = InfoStruct()
        _check(self.lib, self.lib.tslov_tridiag_sign(self.handle, k, a, b, g, _ptr(c), ctypes.byref(info)))
        return c, Info.of(info)

    def block_sign(self, nu: int, site: int, X, x2: torch.Tensor, k: int, x1: torch.Tensor | None = None,
                   defl: "Deflation | None" = None):
        """TSL_k on B = [[H, dH], [0, H]] for U_nu(site) -> exp(i t X) U_nu(site) from (x1, x2)
        (x1 None: zero), optionally deflated by eigenpairs of H (App. E); returns
        (y1, y2, Info): with x1 None, y1 ~ d sgn(H) x2 / dt."""
        import numpy as np
        x2 = self._spinor(x2, "x2")
        x1 = None if x1 is None else self._spinor(x1, "x1")
        Xa = np.ascontiguousarray(np.asarray(X, dtype=np.complex128).reshape(3, 3))
        y1, y2 = self._new_spinor(), self._new_spinor()
        info = InfoStruct()
        Xp = Xa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if defl is None:
            st = self.lib.tslov_block_sign(self.handle, int(nu), int(site), Xp, _ptr(x1), _ptr(x2), int(k), _ptr(y1),
                                           _ptr(y2), ctypes.byref(info))
        else:
            st = self.lib.tslov_block_sign_deflated(self.handle, int(nu), int(site), Xp, _ptr(x1), _ptr(x2), int(k),
                                                    ctypes.byref(defl.struct), _ptr(y1), _ptr(y2), ctypes.byref(info))
        _check(self.lib, st)
        return y1, y2, Info.of(info)

    def block_error_estimate(self, nu: int, site: int, X, psi: torch.Tensor, k: int,
                             defl: "Deflation | None" = None) -> float:
        """eps_B of the block process for the link parameter (eq. bA_error_est), optionally
        with the deflated block process applied twice (App. E)."""
        import numpy as np
        psi = self._spinor(psi, "psi")
        Xa = np.ascontiguousarray(np.asarray(X, dtype=np.complex128).reshape(3, 3))
        eps = ctypes.c_double()
        Xp = Xa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if defl is None:
            st = self.lib.tslov_block_error_estimate(self.handle, int(nu), int(site), Xp, _ptr(psi), int(k),
                                                     ctypes.byref(eps))
        else:
            st = self.lib.tslov_block_error_estimate_deflated(self.handle, int(nu), int(site), Xp, _ptr(psi), int(k),
                                                              ctypes.byref(defl.struct), ctypes.byref(eps))
        _check(self.lib, st)
        return eps.value

    def tune_k(self, k_outer, k_inner=None, trial_target: float = 1e-9, defl: "Deflation | None" = None,
               direction=None, rand: torch.Tensor | None = None):
        """The tuning run of the Krylov sizes on the trial vector (1, ..., 1): dict with
        eps and ms per candidate, chosen (index or -1) and cross (the error of each
        vector of rand, (nrand, V, 4, 3), at the chosen sizes).  direction = (nu, site, X)
        switches to eps_B of the block-matrix derivative."""
        import numpy as np
        n = len(k_outer)
        ko = (ctypes.c_int * n)(*[int(k) for k in k_outer])
        ki = None if k_inner is None else (ctypes.c_int * n)(*[int(k) for k in k_inner])
        eps = (ctypes.c_double * n)()
        ms = (ctypes.c_double * n)()
        chosen = ctypes.c_int()
        d = None if defl is None else ctypes.byref(defl.struct)
        dirp = None
        if direction is not None:
            nu, site, X = direction
            Xa = np.ascontiguousarray(np.asarray(X, dtype=np.complex128)).view(np.float64).ravel()
            dirp = ctypes.byref(LinkDirection(int(nu), int(site), (ctypes.c_double * 18)(*Xa.tolist())))
        nrand, rp, cross = 0, None, None
        if rand is not None:
            rand = self._sources(rand, "rand")
            nrand = rand.shape[0]
            rp = _ptr(rand)
            cross = (ctypes.c_double * nrand)()
        _check(self.lib, self.lib.tslov_tune_k(self.handle, n, ko, ki, float(trial_target), d, dirp, nrand, rp, eps, ms,
                                               ctypes.byref(chosen), cross))
        return {"eps": list(eps), "ms": list(ms), "chosen": chosen.value,
                "cross": list(cross) if (cross is not None and chosen.value >= 0) else []}

    def overlap_solve(self, b: torch.Tensor, k: int, adjoint: bool = False, tol: float = 1e-10, maxit: int = 500):
        """x = D_ov^{-1} b (or D_ov^{-dag} b) with the size-k sign; returns (x, iterations, relative residual)."""
        b = self._spinor(b, "b")
        x = self._new_spinor()
        it, rel = ctypes.c_int(), ctypes.c_double()
        _check(self.lib, self.lib.tslov_overlap_solve(self.handle, _ptr(b), _ptr(x), int(k), int(bool(adjoint)),
                                                      float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rel)))
        return x, it.value, rel.value

    def physical_current(self, xi: torch.Tensor, k: int, tol: float = 1e-10, maxit: int = 500):
        """The Z2-noise estimate of Tr(D_ov^{-1} dD_ov/dTheta) over the sources xi (nsrc, V, 4, 3):
        dict with j (complex (4, V)), div and tot (complex (V,)), iters and relres per source."""
        xi = self._sources(xi, "xi")
        n, V = xi.shape[0], self.volume
        j = torch.empty((2, 4, V), dtype=torch.float64, device=self.device)
        div = torch.empty((2, V), dtype=torch.float64, device=self.device)
        tot = torch.empty((2, V), dtype=torch.float64, device=self.device)
        it, rel = (ctypes.c_int * n)(), (ctypes.c_double * n)()
        _check(self.lib, self.lib.tslov_physical_current(self.handle, n, _ptr(xi), int(k), float(tol), int(maxit),
                                                         _ptr(j), _ptr(div), _ptr(tot), it, rel))
        return {"j": torch.complex(j[0], j[1]), "div": torch.complex(div[0], div[1]),
                "tot": torch.complex(tot[0], tot[1]), "iters": list(it), "relres": list(rel)}

    def set_nested(self, k_inner: int = 0):
        """Nested projected-matrix step of the sign calls with inner Krylov size k_inner (0: plain)."""
        _check(self.lib, self.lib.tslov_set_nested(self.handle, int(k_inner)))

    def set_diagnostics(self, flags: int = 0):
        """DIAG_EPS_A: single-source calls also fill Info.eps_A (one more Lanczos process)."""
        _check(self.lib, self.lib.tslov_set_diagnostics(self.handle, int(flags)))

    def dense_sign(self, T: torch.Tensor, E: torch.Tensor | None = None):
        k = T.shape[0]
        T = T.to(self.device, torch.complex128).contiguous()
        E = None if E is None else E.to(self.device, torch.complex128).contiguous()
        S = torch.empty_like(T)
        L = torch.empty_like(T) if E is not None else None
        it = ctypes.c_int()
        _check(self.lib, self.lib.tslov_dense_sign(self.handle, _ptr(T), int(k), _ptr(E), _ptr(S), _ptr(L),
                                                   ctypes.byref(it)))
        return S, L, it.value

    def timing_enable(self, every: int = 1):
        """Time every `every`-th launch of each kernel class (0 or False: off)."""
        _check(self.lib, self.lib.tslov_timing_enable(self.handle, int(every)))

    def timing_read(self, which: int):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        _check(self.lib, self.lib.tslov_timing_read(self.handle, int(which), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def kernel_bytes(self, which: int) -> float:
        return float(self.lib.tslov_kernel_bytes(self.handle, int(which)))

    def set_graphs(self, on: bool = True):
        """Capture the Lanczos loops as HIP graphs and replay them (needs a non-null stream)."""
        _check(self.lib, self.lib.tslov_set_graphs(self.handle, int(bool(on))))

    def set_apply_chunk(self, T: int = 0):
        """t-slices per chunk of the marching operator (0: timed pick on the first call)."""
        _check(self.lib, self.lib.tslov_set_apply_chunk(self.handle, int(T)))

    def apply_chunk(self) -> int:
        """The timed chunk length of the marching operator (0: none yet, or not marching)."""
        t = ctypes.c_int()
        _check(self.lib, self.lib.tslov_get_apply_chunk(self.handle, ctypes.byref(t)))
        return t.value

    def set_pair_ns(self, ns: int = 0):
        """Entries per workgroup of the batched colour-split pair kernels (0: timed pick)."""
        _check(self.lib, self.lib.tslov_set_pair_ns(self.handle, int(ns)))

    def set_cg_operator(self, form: int = 3):
        """Operator form of the deflated derivative's shifted solves: 0 multi-right-hand-side,
        1 colour split, 2 matrix-core products, 3 t-march (default)."""
        _check(self.lib, self.lib.tslov_set_cg_operator(self.handle, int(form)))

    def pair_ns(self):
        """The timed picks (forward, reverse); 0 while none is made."""
        f, b = ctypes.c_int(), ctypes.c_int()
        _check(self.lib, self.lib.tslov_get_pair_ns(self.handle, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value


def _tridiag_arrays(diag, sub, sup):
    import numpy as np
    d = np.ascontiguousarray(np.asarray(diag, dtype=np.complex128))
    k = d.shape[0]
    lo = np.ascontiguousarray(np.asarray(sub, dtype=np.float64).reshape(max(k - 1, 0)))
    hi = np.ascontiguousarray(np.asarray(sup, dtype=np.complex128).reshape(max(k - 1, 0)))
    keep = (d, lo, hi)
    ptr = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    arrays = (ptr(d), ptr(lo) if k > 1 else None, ptr(hi) if k > 1 else None)
    _tridiag_arrays.keep = keep   # alive until the next call
    return arrays


def ritz_values(diag, sub, sup):
    """Eigenvalues of the tridiagonal T (host, no device needed) and the sweeps used."""
    import numpy as np
    lib = load_library()
    k = len(diag)
    a, b, g = _tridiag_arrays(diag, sub, sup)
    out = np.zeros(2 * k)
    sw = ctypes.c_int()
    _check(lib, lib.tslov_ritz_values(k, a, b, g, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(sw)))
    return out[0::2] + 1j * out[1::2], sw.value


class Deflation:
    """Keeps the eigenvector tensors and the eigenvalue array alive for the C struct."""

    def __init__(self, ctx: Context, R: torch.Tensor, L: torch.Tensor, lam):
        l = int(R.shape[0])
        shape = (l, ctx.volume, 4, 3)
        for t, n in ((R, "R"), (L, "L")):
            if t.dtype != torch.complex128 or t.device != ctx.device or tuple(t.shape) != shape:
                raise ValueError(f"{n} must be complex128 of shape {shape} on {ctx.device}")
        self.R = R.contiguous()
        self.L = L.contiguous()
        lam = [complex(z) for z in lam]
        if len(lam) != l:
            raise ValueError("need one eigenvalue per eigenvector pair")
        self.lam = (ctypes.c_double * (2 * l))(*[v for z in lam for v in (z.real, z.imag)])
        self.struct = DeflationStruct(l, _ptr(self.R), _ptr(self.L), self.lam)


class SignGrad(torch.autograd.Function):
    """S = Re <eta | TSL_k(H(U), psi)> (or, with overlap=True, S = Re <eta | D_ov | psi>)
    with a hand-written backward (HIP).

    ``forward(U, psi, eta, ctx, k, recompute=0, defl=None, overlap=False)`` loads U
    into the context, runs the forward pass and the reverse-mode recursion once
    (regenerating the Krylov vectors in segments of ``recompute`` steps if it is
    positive; deflating by ``defl``, a ``Deflation`` of eigenpairs of H(U), whose
    motion with U is part of the derivative), and keeps dS/dU, dS/dpsi and
    dS/deta (= the output TSL_k(psi), resp. D_ov psi).  ``backward`` scales them
    by the incoming gradient (torch's convention for real outputs of complex
    inputs: grad = dS/dRe + i dS/dIm).  The eigenpair tensors get no gradient:
    they are functions of U, and their dependence is inside dS/dU.
    """

    @staticmethod
    def forward(ctx, U, psi, eta, context: Context, k: int, recompute: int = 0, defl: "Deflation | None" = None,
                overlap: bool = False):
        context.set_links(U.detach())
        if overlap:
            S, dU, dpsi, deta, _ = context.overlap_grad(eta.detach(), psi.detach(), k, defl=defl,
                                                        recompute=recompute)
        else:
            S, dU, dpsi, _, deta = context.sign_grad(eta.detach(), psi.detach(), k, want_dpsi=True, defl=defl,
                                                     recompute=recompute, want_y=True)
        ctx.save_for_backward(dU, dpsi, deta)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad):
        dU, dpsi, deta = ctx.saved_tensors
        return grad * dU, grad * dpsi, grad * deta, None, None, None, None, None
