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
_lib.lupp_timing_bytes.argtypes = [_vp, _i32, ctypes.POINTER(ctypes.c_double)]
_lib.lupp_workspace_bytes.argtypes = [_vp, _i32, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)]
_lib.lupp_test_inject_fault.argtypes = [_vp, _i32]
_lib.lupp_status_string.argtypes = [_i32]
_lib.lupp_status_string.restype = ctypes.c_char_p
for _name in ("lupp_dgetrf", "lupp_sgetrf"):
    getattr(_lib, _name).argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp]
_lib.lupp_dgeqrf.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp]
_lib.lupp_drandutv.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_int32, _vp, _i64, _vp, _i64, _vp, _i64]
for _name in ("lupp_dgetrs", "lupp_sgetrs"):
    getattr(_lib, _name).argtypes = [_vp, _char, _i64, _i64, _vp, _i64, _vp, _vp, _i64]

OPT_NB = 1
OPT_PANEL_LEAF = 2
OPT_TIMING = 3
OPT_LOOKAHEAD = 4
OPT_UPDATE_PREC = 5
OPT_DEFER_SWAPS = 6
OPT_SPLIT_UPDATE = 7
OPT_LP_PACKED = 8
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "fp8": 3}
IR_SOLVER = {"classical": 0, "gmres": 1}
IR_STATUS = {0: "converged", 1: "stagnated", 2: "diverged", 3: "singular", 4: "maxiter"}
ERR_INTERNAL = 2001
ERR_UNSUPPORTED = 2002
ERR_SINGULAR = 2003
WS = {"dgetrf": 1, "sgetrf": 2, "dgetrs": 3, "sgetrs": 4, "dgesv_mixed": 5, "batched": 6}


class IrOpts(ctypes.Structure):
    """lupp_ir_opts (field order and types as in include/lupp.h)."""
    _fields_ = [("factor_prec", ctypes.c_int32), ("solver", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("gmres_restart", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("nb", ctypes.c_int64), ("fallback_fp64", ctypes.c_int32)]


class IrReport(ctypes.Structure):
    """lupp_ir_report."""
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("info", ctypes.c_int32), ("fallback_used", ctypes.c_int32), ("backward_error", ctypes.c_double),
                ("factor_ms", ctypes.c_double), ("refine_ms", ctypes.c_double)]


_lib.lupp_ir_opts_default.argtypes = [ctypes.POINTER(IrOpts), ctypes.c_int32]
_lib.lupp_ir_opts_default.restype = None
_lib.lupp_dgesv_mixed.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(IrOpts),
                                  ctypes.POINTER(IrReport)]
for _name in ("lupp_dgesv_batched", "lupp_sgesv_batched", "lupp_dgesv_batched_noalloc"):
    getattr(_lib, _name).argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
for _name in ("lupp_dgetrf_batched", "lupp_sgetrf_batched"):
    getattr(_lib, _name).argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
BATCH_MAX_N = 128
BATCH_MAX_CLASSES = 6


class BatchedSchedule(ctypes.Structure):
    """lupp_batched_schedule."""
    _fields_ = [("nclass", ctypes.c_int32), ("nmax", ctypes.c_int32 * BATCH_MAX_CLASSES),
                ("shape", ctypes.c_int32 * BATCH_MAX_CLASSES), ("grid_pct", ctypes.c_int32 * BATCH_MAX_CLASSES)]


_i32p = ctypes.POINTER(ctypes.c_int32)
_lib.lupp_batched_shape_count.argtypes = []
_lib.lupp_batched_shape.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, _i32p]
_lib.lupp_batched_get_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(BatchedSchedule)]
_lib.lupp_batched_set_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(BatchedSchedule)]


def batched_shapes() -> list[dict]:
    """The compiled kernel shapes of the batched path (host only)."""
    out = []
    for v in range(_lib.lupp_batched_shape_count()):
        nw, rows, cols, nmax = (ctypes.c_int32() for _ in range(4))
        _check(_lib.lupp_batched_shape(v, ctypes.byref(nw), ctypes.byref(rows), ctypes.byref(cols),
                                       ctypes.byref(nmax)), "lupp_batched_shape")
        out.append({"wavefronts": nw.value, "rows": rows.value, "cols": cols.value, "nmax": nmax.value})
    return out


def _sched_to_dict(s: BatchedSchedule) -> dict:
    k = s.nclass
    return {"nclass": k, "nmax": list(s.nmax[:k]), "shape": list(s.shape[:k]), "grid_pct": list(s.grid_pct[:k])}


def _sched_from_dict(d: dict) -> BatchedSchedule:
    s = BatchedSchedule()
    s.nclass = int(d["nclass"])
    for c in range(min(max(s.nclass, 0), BATCH_MAX_CLASSES)):  # the library validates nclass
        s.nmax[c] = int(d["nmax"][c])
        s.shape[c] = int(d["shape"][c])
        s.grid_pct[c] = int(d["grid_pct"][c])
    return s
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

    def __init__(self, tuned: bool = True):
        """tuned: install the cached batched schedules of this device's
        architecture (paper_2104_05782_amd/autotune.py), if any."""
        p = _vp()
        _check(_lib.lupp_create(ctypes.byref(p)), "lupp_create")
        self._p = p
        self.device = torch.cuda.current_device()
        if tuned:
            from .autotune import apply_cached
            apply_cached(self)

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

    def workspace_bytes(self, op: str, m: int = 0, n: int = 0, k: int = 0) -> int:
        """lupp_workspace_bytes for a call kind of WS."""
        out = ctypes.c_size_t()
        _check(_lib.lupp_workspace_bytes(self._p, WS[op], m, n, k, ctypes.byref(out)), "lupp_workspace_bytes")
        return out.value

    def inject_fault(self, what: int):
        """lupp_test_inject_fault (test hook of lupp_sync's error paths)."""
        _check(_lib.lupp_test_inject_fault(self._p, what), "lupp_test_inject_fault")

    def batched_schedule(self, dtype: str) -> dict:
        """The handle's batched schedule for "f64" or "f32"."""
        s = BatchedSchedule()
        _check(_lib.lupp_batched_get_schedule(self._p, int(dtype == "f32"), ctypes.byref(s)),
               "lupp_batched_get_schedule")
        return _sched_to_dict(s)

    def set_batched_schedule(self, dtype: str, sched: dict | None):
        """Install a schedule (dict as returned by batched_schedule); None
        restores the initial one."""
        s = _sched_from_dict(sched) if sched is not None else None
        _check(_lib.lupp_batched_set_schedule(self._p, int(dtype == "f32"), ctypes.byref(s) if s else None),
               "lupp_batched_set_schedule")

    def timing_bytes(self, phase: str) -> float:
        """Summed algorithmic bytes recorded for a phase (lupp_timing_bytes)."""
        b = ctypes.c_double()
        _check(_lib.lupp_timing_bytes(self._p, PHASES[phase], ctypes.byref(b)), "lupp_timing_bytes")
        return b.value

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


def ir_opts(solver: str = "gmres", **kw) -> IrOpts:
    """lupp_ir_opts with the library defaults for `solver`, then the keyword overrides
    (factor_prec accepts a name of PREC)."""
    o = IrOpts()
    _lib.lupp_ir_opts_default(ctypes.byref(o), IR_SOLVER[solver])
    for k, v in kw.items():
        if k == "factor_prec" and isinstance(v, str):
            v = PREC[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def lupp_dgesv_mixed(A, B, X, opts: IrOpts | None = None, handle: Handle | None = None) -> dict:
    """X := solution of A X = B by the mixed-precision factorization and FP64
    refinement (A, B, X float64 column-major device matrices; A and B are not
    modified).  Returns the report as a dict."""
    _dev(A, torch.float64, "A")
    _dev(B, torch.float64, "B")
    _dev(X, torch.float64, "X")
    n = A.shape[0]
    if A.shape[1] != n or B.shape[0] != n or tuple(X.shape) != tuple(B.shape):
        raise ValueError("A must be n x n, B and X n x nrhs")
    h = _prep(handle)
    rep = IrReport()
    o = opts if opts is not None else ir_opts()
    _check(_lib.lupp_dgesv_mixed(h.ptr, n, B.shape[1], A.data_ptr(), _lead(A), B.data_ptr(), _lead(B), X.data_ptr(),
                                 _lead(X), ctypes.byref(o), ctypes.byref(rep)), "lupp_dgesv_mixed")
    out = {f: getattr(rep, f) for f, _ in IrReport._fields_}
    out["status_name"] = IR_STATUS.get(rep.status, "unknown")
    return out


def gesv_mixed(A: torch.Tensor, B: torch.Tensor, handle: Handle | None = None, solver: str = "gmres", **kw):
    """Solve A X = B (B a matrix or a vector) with lupp_dgesv_mixed; returns (X, report)."""
    B2 = B if B.dim() == 2 else B.view(-1, 1)
    X = torch.empty(B2.shape[1], B2.shape[0], dtype=torch.float64, device=B.device).t()
    rep = lupp_dgesv_mixed(A, colmajor(B2), X, ir_opts(solver, **kw), handle)
    return (X if B.dim() == 2 else X[:, 0]), rep


def lupp_xgesv_batched(n, A, a_off, ipiv, p_off, B, b_off, info, handle: Handle | None = None):
    """Batched factorization and solve (lupp_dgesv_batched / lupp_sgesv_batched by
    A's dtype): every argument is a device tensor (n int32, offsets int64, ipiv
    and info int32, A and B packed float64/float32); B=None factors only."""
    batch = int(n.numel())
    for t, dt, what in ((n, torch.int32, "n"), (a_off, torch.int64, "a_off"), (p_off, torch.int64, "p_off"),
                        (ipiv, torch.int32, "ipiv"), (info, torch.int32, "info")):
        _dev(t, dt, what)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % what)
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("A must be float64 or float32")
    _dev(A, A.dtype, "A")
    if info.numel() < batch or a_off.numel() < batch or p_off.numel() < batch:
        raise ValueError("n, a_off, p_off and info need one entry per system")
    h = _prep(handle)
    d = A.dtype == torch.float64
    if B is None:
        fn = _lib.lupp_dgetrf_batched if d else _lib.lupp_sgetrf_batched
        _check(fn(h.ptr, batch, n.data_ptr(), a_off.data_ptr(), A.data_ptr(), p_off.data_ptr(), ipiv.data_ptr(),
                  info.data_ptr()), fn.__name__)
        return
    _dev(B, A.dtype, "B")
    _dev(b_off, torch.int64, "b_off")
    if b_off.numel() < batch:
        raise ValueError("b_off needs one entry per system")
    fn = _lib.lupp_dgesv_batched if d else _lib.lupp_sgesv_batched
    _check(fn(h.ptr, batch, n.data_ptr(), a_off.data_ptr(), A.data_ptr(), p_off.data_ptr(), ipiv.data_ptr(),
              b_off.data_ptr(), B.data_ptr(), info.data_ptr()), fn.__name__)


NOALLOC_MAX_BATCH = 1048576


def lupp_dgesv_batched_noalloc(n, A, a_off, ipiv, p_off, B, b_off, info, handle: Handle | None = None):
    """lupp_dgesv_batched_noalloc: lupp_dgesv_batched with the library's fixed
    scratch array instead of handle workspace (FP64, with right-hand sides)."""
    batch = int(n.numel())
    for t, dt, what in ((n, torch.int32, "n"), (a_off, torch.int64, "a_off"), (p_off, torch.int64, "p_off"),
                        (ipiv, torch.int32, "ipiv"), (info, torch.int32, "info"), (A, torch.float64, "A"),
                        (B, torch.float64, "B"), (b_off, torch.int64, "b_off")):
        _dev(t, dt, what)
    if min(info.numel(), a_off.numel(), p_off.numel(), b_off.numel()) < batch:
        raise ValueError("n, a_off, p_off, b_off and info need one entry per system")
    h = _prep(handle)
    fn = _lib.lupp_dgesv_batched_noalloc
    _check(fn(h.ptr, batch, n.data_ptr(), a_off.data_ptr(), A.data_ptr(), p_off.data_ptr(), ipiv.data_ptr(),
              b_off.data_ptr(), B.data_ptr(), info.data_ptr()), fn.__name__)


def gesv_batched(n, A, a_off, B=None, b_off=None, handle: Handle | None = None):
    """Factor (and solve, when B is given) the packed batch in place; returns
    (ipiv, p_off, info) device tensors (p_off: exclusive prefix sums of n)."""
    n64 = n.to(torch.int64)
    p_off = torch.zeros_like(n64)
    if n.numel() > 1:
        p_off[1:] = torch.cumsum(n64, 0)[:-1]
    ipiv = torch.zeros(max(1, int(n64.clamp(min=0).sum().item())), dtype=torch.int32, device=A.device)
    info = torch.zeros(max(1, n.numel()), dtype=torch.int32, device=A.device)
    lupp_xgesv_batched(n, A, a_off, ipiv, p_off, B, b_off, info, handle)
    return ipiv, p_off, info


def lupp_dgeqrf(A, tau, handle: Handle | None = None):
    """Householder QR in place of column-major float64 A; tau float64[min(m, n)]."""
    _dev(A, torch.float64, "A")
    _dev(tau, torch.float64, "tau")
    m, n = A.shape
    if tau.numel() < min(m, n):
        raise ValueError("tau needs min(m, n) entries")
    h = _prep(handle)
    _check(_lib.lupp_dgeqrf(h.ptr, m, n, A.data_ptr(), _lead(A), tau.data_ptr()), "lupp_dgeqrf")


def geqrf(A: torch.Tensor, handle: Handle | None = None) -> torch.Tensor:
    """Factor column-major float64 A in place (R above, Householder vectors
    below the diagonal); returns tau."""
    m, n = A.shape
    tau = torch.empty(max(1, min(m, n)), dtype=torch.float64, device=A.device)
    lupp_dgeqrf(A, tau, handle)
    return tau[:min(m, n)]


def lupp_drandutv(A, G, q: int, U=None, V=None, handle: Handle | None = None):
    """randUTV in place of column-major float64 A (n x n) -> T; U and V
    (column-major n x n float64, or None) receive the orthogonal factors; G
    (n x n) holds the Gaussian draws."""
    n = A.shape[0]
    _dev(A, torch.float64, "A")
    _dev(G, torch.float64, "G")
    if A.shape != (n, n) or G.shape[0] < n or G.shape[1] < n:
        raise ValueError("A must be n x n and G at least n x n")
    for X, what in ((U, "U"), (V, "V")):
        if X is not None:
            _dev(X, torch.float64, what)
            if X.shape != (n, n):
                raise ValueError("%s must be n x n" % what)
    h = _prep(handle)
    _check(_lib.lupp_drandutv(h.ptr, n, A.data_ptr(), _lead(A), int(q), G.data_ptr(), _lead(G),
                              U.data_ptr() if U is not None else None, _lead(U) if U is not None else 1,
                              V.data_ptr() if V is not None else None, _lead(V) if V is not None else 1),
           "lupp_drandutv")


def randutv(A: torch.Tensor, G: torch.Tensor, q: int = 1, handle: Handle | None = None):
    """(U, T, V) of A = U T V^T (A is overwritten by T and returned as T)."""
    n = A.shape[0]
    U = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
    V = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
    lupp_drandutv(A, G, q, U, V, handle)
    return U, A, V


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
