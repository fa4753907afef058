"""CPU oracle for LU with partial pivoting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path:
the arithmetic lives in ``lupp_oracle.c`` (plain C, FP64 and FP32, compiled
with gcc ``-O2 -ffp-contract=off``), loaded here through ctypes.  The checkers
in ``checks.py`` compute the acceptance measures (scaled residual, backward
error) from their definitions with numpy.

The method and its conventions are stated in the header of ``lupp_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lupp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, ip = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        for name in ("oracle_dgetrf", "oracle_sgetrf"):
            f = getattr(lib, name)
            f.argtypes = [i64, i64, ip, i64, ip, ip, i64, i32]
            f.restype = i32
        lib.oracle_dgetrf_left.argtypes = [i64, i64, ip, i64, ip]
        lib.oracle_dgetrf_left.restype = i32
        for name in ("oracle_dgetrs", "oracle_sgetrs"):
            f = getattr(lib, name)
            f.argtypes = [i64, i64, ip, i64, ip, ip, i64]
            f.restype = i32
        for name in ("oracle_dgesv_batched", "oracle_sgesv_batched"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int32, ip, ip, ip, ip, ip, ip, ip, ip, i32]
            f.restype = None
        lib.oracle_max_threads.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def host_cores() -> int:
    """Cores this process may run on (affinity mask)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def getrf(A: np.ndarray, ksteps: int = -1, nthreads: int = 1, with_gap: bool = False, overwrite: bool = False):
    """Factor a copy of A (FP64 or FP32).  Returns (LU, ipiv, info[, gap]).

    ``ksteps >= 0`` stops after that many elimination steps (the array then
    holds the factored leading part and the Schur complement).  With
    ``overwrite`` a writable Fortran-ordered FP64/FP32 A is factored in place
    (no copy; used when the copy must stay outside a timed interval).
    """
    if not (overwrite and isinstance(A, np.ndarray) and A.flags["F_CONTIGUOUS"] and A.flags["WRITEABLE"]
            and A.dtype in (np.float64, np.float32)):
        A = np.array(A, order="F", copy=True)
    if A.dtype not in (np.float64, np.float32):
        A = A.astype(np.float64, order="F")
    m, n = A.shape
    p = min(m, n)
    ipiv = np.zeros(p, dtype=np.int32)
    gap = np.zeros(p, dtype=np.float64)
    fn = _load().oracle_dgetrf if A.dtype == np.float64 else _load().oracle_sgetrf
    info = fn(m, n, _ptr(A), max(m, 1), _ptr(ipiv), _ptr(gap), ksteps, nthreads)
    if ksteps >= 0 and ksteps < p:
        ipiv, gap = ipiv[:ksteps], gap[:ksteps]
    return (A, ipiv, info, gap) if with_gap else (A, ipiv, info)


def getrf_left(A: np.ndarray):
    """Left-looking FP64 variant (bitwise identical by construction)."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    ipiv = np.zeros(min(m, n), dtype=np.int32)
    info = _load().oracle_dgetrf_left(m, n, _ptr(A), max(m, 1), _ptr(ipiv))
    return A, ipiv, info


def getrs(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray):
    """Solve with the factors; returns (X, status) -- status = first zero U(k,k)."""
    LU = np.asfortranarray(LU)
    n = LU.shape[0]
    X = np.array(B, dtype=LU.dtype, order="F", copy=True)
    vec = X.ndim == 1
    if vec:
        X = X.reshape(n, 1, order="F")
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    fn = _load().oracle_dgetrs if LU.dtype == np.float64 else _load().oracle_sgetrs
    st = fn(n, X.shape[1], _ptr(LU), max(n, 1), _ptr(ipiv), _ptr(X), max(n, 1))
    return (X.ravel() if vec else X), st


def gesv_batched(nvec, A_packed, a_off, B_packed, b_off, nthreads: int | None = None):
    """Factor and solve every packed system.  Returns (LU, ipiv, p_off, X, info)."""
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    A = np.array(A_packed, copy=True)
    B = np.array(B_packed, dtype=A.dtype, copy=True)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    p_off = np.zeros(len(nvec), dtype=np.int64)
    if len(nvec):
        p_off[1:] = np.cumsum(nvec.astype(np.int64))[:-1]
    ipiv = np.zeros(int(nvec.astype(np.int64).sum()), dtype=np.int32)
    info = np.zeros(len(nvec), dtype=np.int32)
    fn = _load().oracle_dgesv_batched if A.dtype == np.float64 else _load().oracle_sgesv_batched
    fn(len(nvec), _ptr(nvec), _ptr(a_off), _ptr(A), _ptr(p_off), _ptr(ipiv), _ptr(b_off),
       _ptr(B), _ptr(info), nthreads or host_cores())
    return A, ipiv, p_off, B, info


def max_threads() -> int:
    return _load().oracle_max_threads()
