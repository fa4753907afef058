"""ctypes binding of liblupp.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblupp.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("liblupp.so is not built (run: python -m paper_2104_05782_amd.build); "
                      "there is no fallback implementation")
_lib = ctypes.CDLL(LIB_PATH)

_i64, _i32, _vp, _char = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_char
_lib.lupp_create.argtypes = [ctypes.POINTER(_vp)]
_lib.lupp_destroy.argtypes = [_vp]
_lib.lupp_set_stream.argtypes = [_vp, _vp]
_lib.lupp_set_option.argtypes = [_vp, _i32, _i64]
_lib.lupp_sync.argtypes = [_vp]
_lib.lupp_timing_summary.argtypes = [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), _i32]
_lib.lupp_status_string.argtypes = [_i32]
_lib.lupp_status_string.restype = ctypes.c_char_p
for _name in ("lupp_dgetrf", "lupp_sgetrf"):
    getattr(_lib, _name).argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp]
for _name in ("lupp_dgetrs", "lupp_sgetrs"):
    getattr(_lib, _name).argtypes = [_vp, _char, _i64, _i64, _vp, _i64, _vp, _vp, _i64]

OPT_NB = 1
OPT_PANEL_LEAF = 2
OPT_TIMING = 3
PHASES = {"panel": 0, "laswp": 1, "trsm": 2, "update": 3, "update_big": 4, "panel_leaf": 5, "panel_swap": 6,
          "panel_trsm": 7, "panel_gemm": 8}


class LuppError(RuntimeError):
    def __init__(self, rc: int, where: str):
        super().__init__("%s: %s (%d)" % (where, status_string(rc), rc))
        self.rc = rc


def status_string(rc: int) -> str:
    return _lib.lupp_status_string(rc).decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise LuppError(rc, where)


class Handle:
    """Owns a lupp handle (workspace) on the current device."""

    def __init__(self):
        p = _vp()
        _check(_lib.lupp_create(ctypes.byref(p)), "lupp_create")
        self._p = p
        self.device = torch.cuda.current_device()

    @property
    def ptr(self):
        return self._p

    def set_stream(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.lupp_set_stream(self._p, _vp(s.cuda_stream)), "lupp_set_stream")

    def set_option(self, option: int, value: int):
        _check(_lib.lupp_set_option(self._p, option, value), "lupp_set_option")

    def sync(self):
        _check(_lib.lupp_sync(self._p), "lupp_sync")

    def timing_summary(self, phase: str, reset: bool = False):
        """(count, ms, flops) recorded for a phase (see lupp_timing_summary)."""
        c, ms, fl = _i64(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.lupp_timing_summary(self._p, PHASES[phase], ctypes.byref(c), ctypes.byref(ms), ctypes.byref(fl),
                                        int(reset)), "lupp_timing_summary")
        return c.value, ms.value, fl.value

    def close(self):
        if getattr(self, "_p", None):
            _lib.lupp_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def default_handle() -> Handle:
    dev = torch.cuda.current_device()
    h = _handles.get(dev)
    if h is None:
        h = _handles[dev] = Handle()
    return h


def colmajor(A: torch.Tensor) -> torch.Tensor:
    """Column-major copy (or A itself when already column-major)."""
    if A.dim() != 2:
        raise ValueError("expected a matrix")
    if A.stride(0) == 1 and (A.shape[1] <= 1 or A.stride(1) >= max(1, A.shape[0])):
        return A
    return A.t().contiguous().t()


def _lead(A: torch.Tensor) -> int:
    m, n = A.shape
    if m > 1 and A.stride(0) != 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    return max(1, m) if n <= 1 else A.stride(1)


def _dev(t: torch.Tensor, dtype, what: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (what, dtype))


def _prep(handle):
    h = handle or default_handle()
    h.set_stream()
    return h


def _getrf(fn, dtype, A, ipiv, info, handle):
    _dev(A, dtype, "A")
    _dev(ipiv, torch.int32, "ipiv")
    _dev(info, torch.int32, "info")
    m, n = A.shape
    if ipiv.numel() < min(m, n) or not ipiv.is_contiguous():
        raise ValueError("ipiv needs min(m, n) contiguous int32 entries")
    h = _prep(handle)
    _check(fn(h.ptr, m, n, A.data_ptr(), _lead(A), ipiv.data_ptr(), info.data_ptr()), fn.__name__)


def lupp_dgetrf(A, ipiv, info, handle: Handle | None = None):
    """In-place P*A = L*U of a column-major float64 device matrix."""
    _getrf(_lib.lupp_dgetrf, torch.float64, A, ipiv, info, handle)


def lupp_sgetrf(A, ipiv, info, handle: Handle | None = None):
    """In-place P*A = L*U of a column-major float32 device matrix."""
    _getrf(_lib.lupp_sgetrf, torch.float32, A, ipiv, info, handle)


def _getrs(fn, dtype, LU, ipiv, B, handle):
    _dev(LU, dtype, "LU")
    _dev(B, dtype, "B")
    _dev(ipiv, torch.int32, "ipiv")
    n = LU.shape[0]
    if LU.shape[1] != n or B.shape[0] != n:
        raise ValueError("LU must be n x n and B n x nrhs")
    h = _prep(handle)
    _check(fn(h.ptr, b"N", n, B.shape[1], LU.data_ptr(), _lead(LU), ipiv.data_ptr(), B.data_ptr(), _lead(B)),
           fn.__name__)


def lupp_dgetrs(LU, ipiv, B, handle: Handle | None = None):
    """B := inv(A) * B from the float64 factors (B column-major, in place)."""
    _getrs(_lib.lupp_dgetrs, torch.float64, LU, ipiv, B, handle)


def lupp_sgetrs(LU, ipiv, B, handle: Handle | None = None):
    """B := inv(A) * B from the float32 factors (B column-major, in place)."""
    _getrs(_lib.lupp_sgetrs, torch.float32, LU, ipiv, B, handle)


def getrf(A: torch.Tensor, handle: Handle | None = None):
    """Factor column-major A in place; returns (ipiv, info) device tensors."""
    m, n = A.shape
    ipiv = torch.empty(max(1, min(m, n)), dtype=torch.int32, device=A.device)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    (lupp_dgetrf if A.dtype == torch.float64 else lupp_sgetrf)(A, ipiv, info, handle)
    return ipiv[:min(m, n)], info


def getrs(LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, handle: Handle | None = None):
    """Solve in place of B (column-major, or a vector); returns B."""
    B2 = B if B.dim() == 2 else B.view(-1, 1)
    (lupp_dgetrs if LU.dtype == torch.float64 else lupp_sgetrs)(LU, ipiv, B2, handle)
    return B
