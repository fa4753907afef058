"""Seeded synthetic inputs for the LU-with-partial-pivoting path.

This module is shared by the CPU oracle side and the GPU side.  It draws and
arranges random numbers only; it contains none of the factorization's
arithmetic.  Every matrix is returned column-major (numpy ``order="F"``).

Generator: numpy's Philox-4x64-10 counter-based bit generator (Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by
``key = (stream_id << 64) | seed``.  Element ``(i, j)`` of an ``m x n`` matrix
drawn from one stream is draw number ``j*m + i`` of that stream.

* ``U(0,1)``  = (top 53 bits of a 64-bit draw) * 2^-53 (numpy ``random()``).
* ``U(-1,1)`` = 2u - 1 and ``U(-0.5,0.5)`` = u - 0.5; both maps are exact in
  binary64.
* FP32 inputs are the round-to-nearest-even conversion of the FP64 draw.

The paper measures on randomly generated dense matrices (its performance
section); these recipes stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

DEFAULT_SEED = 20210512

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "philox.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the threaded Philox fill (philox.c) into synth/libsynth.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _fast():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, vp, i64, c_int, dbl = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.synth_u01.argtypes = [u64, u64, u64, vp, i64, c_int]
        lib.synth_affine_u01.argtypes = [u64, u64, u64, vp, i64, dbl, dbl, c_int]
        _lib = lib
    return _lib


def _threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return 1


def stream(seed: int, stream_id: int) -> np.random.Generator:
    """Independent Philox stream for (seed, stream_id)."""
    if seed < 0 or seed >= 1 << 64 or stream_id < 0 or stream_id >= 1 << 64:
        raise ValueError("seed and stream_id must fit in 64 bits")
    return np.random.Generator(np.random.Philox(key=(int(stream_id) << 64) | int(seed)))


def _u01_transposed(g: np.random.Generator, m: int, n: int) -> np.ndarray:
    # draw number j*m + i -> element (i, j): fill the transposed C-order array
    buf = np.empty((n, m), dtype=np.float64)
    g.random(out=buf)
    return buf


def uniform(seed: int, stream_id: int, m: int, n: int, lo: float = -1.0, hi: float = 1.0,
            dtype=np.float64) -> np.ndarray:
    """m x n column-major matrix with iid U(lo, hi) entries.

    Only the exact affine maps (-1,1) and (-0.5,0.5) and (0,1) are offered so
    that the FP64 values are exact functions of the 53-bit draws.  Filled by
    philox.c (threaded, same stream as numpy's Philox; see tests).
    """
    maps = {(-1.0, 1.0): (2.0, -1.0), (-0.5, 0.5): (1.0, -0.5), (0.0, 1.0): (1.0, 0.0)}
    if (lo, hi) not in maps:
        raise ValueError("supported ranges: (-1,1), (-0.5,0.5), (0,1)")
    stream(seed, stream_id)  # validates the key
    a, b = maps[(lo, hi)]
    t = np.empty((n, m), dtype=np.float64)
    if t.size:
        _fast().synth_affine_u01(int(seed), int(stream_id), 0, t.ctypes.data, t.size, a, b, _threads())
    if dtype != np.float64:
        t = t.astype(dtype)
    return t.T


def uniform_numpy(seed: int, stream_id: int, m: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Reference path of ``uniform`` through numpy's own Philox generator."""
    t = _u01_transposed(stream(seed, stream_id), m, n)
    if (lo, hi) == (-1.0, 1.0):
        t *= 2.0
        t -= 1.0
    elif (lo, hi) == (-0.5, 0.5):
        t -= 0.5
    elif (lo, hi) != (0.0, 1.0):
        raise ValueError("supported ranges: (-1,1), (-0.5,0.5), (0,1)")
    return t.T


def permutation(seed: int, stream_id: int, n: int) -> np.ndarray:
    """Seeded uniformly random permutation of range(n) (numpy's Fisher-Yates)."""
    return stream(seed, stream_id).permutation(n)


def diag_dominant(seed: int, stream_id: int, n: int, dtype=np.float64) -> np.ndarray:
    """Entries iid U(-0.5, 0.5); then a_ii := sum_j |a_ij| over the whole row
    (the original a_ii included).  Row diagonally dominant."""
    a = uniform(seed, stream_id, n, n, -0.5, 0.5, np.float64)
    d = np.abs(a).sum(axis=1)
    a[np.arange(n), np.arange(n)] = d
    return np.asfortranarray(a.astype(dtype, copy=False))


def pi_times_coldom(seed: int, stream_id: int, n: int, dtype=np.float64):
    """A = Pi * D with D strictly column diagonally dominant by an absolute
    margin of 1: d_ij iid U(-1,1) off the diagonal and
    d_jj = 1 + sum_{i != j} |d_ij|.  Row i of D is placed at row perm[i] of A.

    Returns (A, perm).  Partial pivoting on A selects, at step k, the row that
    holds D's row k (column dominance with a margin survives elimination), so
    the pivots have a closed form in terms of ``perm``.
    """
    d = uniform(seed, stream_id, n, n, -1.0, 1.0, np.float64)
    idx = np.arange(n)
    d[idx, idx] = 0.0
    colsum = np.abs(d).sum(axis=0)
    d[idx, idx] = 1.0 + colsum
    perm = permutation(seed, stream_id + 1, n)
    a = np.empty_like(d, order="F")
    a[perm, :] = d
    return np.asfortranarray(a.astype(dtype, copy=False)), perm


def exact_lu_factors(seed: int, stream_id: int, n: int):
    """Factors of a matrix whose LU factorization is exact in binary32/64.

    * L: unit lower triangular; each strict-lower entry is 0 with probability
      1/2, else one of +-1/2, +-1/4.
    * U: upper triangular, off-diagonal entries in {-2..2}, diagonal in
      {-4,-3,-2,-1,1,2,3,4}.
    * perm: seeded permutation; row i of L*U goes to row perm[i] of A.

    Every partial sum an LU factorization of A = Pi^T L U forms is an integer
    multiple of 1/4 bounded by 4n, hence exact in binary32 for n <= 2^18 and in
    binary64, whatever the summation order.  Because |l_ij| <= 1/2 < 1 = l_ii,
    partial pivoting reproduces perm, L and U exactly.
    """
    g = stream(seed, stream_id)
    lvals = np.array([0.0, 0.0, 0.0, 0.0, 0.5, -0.5, 0.25, -0.25])
    L = np.tril(lvals[g.integers(0, 8, size=(n, n), dtype=np.int8)], -1)
    L[np.arange(n), np.arange(n)] = 1.0
    U = np.triu(g.integers(-2, 3, size=(n, n), dtype=np.int8).astype(np.float64), 1)
    dvals = np.array([-4.0, -3.0, -2.0, -1.0, 1.0, 2.0, 3.0, 4.0])
    U[np.arange(n), np.arange(n)] = dvals[g.integers(0, 8, size=n)]
    perm = permutation(seed, stream_id + 1, n)
    return np.asfortranarray(L), np.asfortranarray(U), perm


def exact_lu_product(seed: int, stream_id: int, n: int, dtype=np.float64):
    """A = Pi^T L U from ``exact_lu_factors`` (product formed here, exactly).

    Returns (A, L, U, perm)."""
    L, U, perm = exact_lu_factors(seed, stream_id, n)
    LU = L @ U  # exact: multiples of 1/4 bounded by 4n
    a = np.empty((n, n), order="F")
    a[perm, :] = LU
    return np.asfortranarray(a.astype(dtype, copy=False)), L, U, perm


def gaussian(seed: int, stream_id: int, m: int, n: int) -> np.ndarray:
    """m x n column-major iid N(0,1) (numpy's ziggurat on the Philox stream)."""
    return np.asfortranarray(stream(seed, stream_id).standard_normal((n, m)).T)


def kappa_matrix(seed: int, n: int, kappa: float, stream_id: int = 2) -> np.ndarray:
    """A = U diag(sigma) V^T, sigma_i = kappa^(-(i-1)/(n-1)), U and V the Q
    factors of QR of iid Gaussian matrices, signs fixed so diag(R) > 0."""
    def haar(sid):
        q, r = np.linalg.qr(gaussian(seed, sid, n, n))
        return q * np.sign(np.diag(r))[None, :]
    u = haar(stream_id)
    v = haar(stream_id + 1)
    sig = kappa ** (-(np.arange(n) / max(n - 1, 1)))
    return np.asfortranarray((u * sig[None, :]) @ v.T)


def batch_sizes(seed: int, count: int, lo: int = 8, hi: int = 128, stream_id: int = 1000) -> np.ndarray:
    """Per-system orders n_i iid uniform integers on [lo, hi]."""
    return stream(seed, stream_id).integers(lo, hi + 1, size=count).astype(np.int32)


def batch_uniform(seed: int, sizes: np.ndarray, dtype=np.float64, stream_base: int = 1 << 20):
    """Packed batch of column-major n_i x n_i matrices and n_i right-hand sides,
    entries iid U(-1,1); system i's A comes from stream (stream_base + 2i) and
    its b from (stream_base + 2i + 1).

    Returns (A_packed, a_off, B_packed, b_off) with int64 element offsets.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    a_off = np.zeros(len(sizes), dtype=np.int64)
    b_off = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes):
        a_off[1:] = np.cumsum(sizes * sizes)[:-1]
        b_off[1:] = np.cumsum(sizes)[:-1]
    A = np.empty(int((sizes * sizes).sum()), dtype=np.float64)
    B = np.empty(int(sizes.sum()), dtype=np.float64)
    for i, n in enumerate(sizes):
        n = int(n)
        A[a_off[i]:a_off[i] + n * n] = uniform(seed, stream_base + 2 * i, n, n).ravel(order="F")
        B[b_off[i]:b_off[i] + n] = uniform(seed, stream_base + 2 * i + 1, n, 1).ravel(order="F")
    return A.astype(dtype, copy=False), a_off, B.astype(dtype, copy=False), b_off
