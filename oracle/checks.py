"""Acceptance measures for LU with partial pivoting -- TEST INFRASTRUCTURE ONLY.

Definitions (FP64 unless stated):

* ``perm_from_ipiv``: the LAPACK sequential-interchange vector (1-based,
  interchange k swaps rows k and ipiv[k]-1) turned into the row permutation p
  with (P A)[i, :] = A[p[i], :].
* ``scaled_residual``: ||P A - L U||_1 / (n * eps * ||A||_1), with L and U
  promoted to FP64 and the product formed in FP64; eps is the unit roundoff of
  the factor precision (2^-53 for FP64 factors, 2^-24 for FP32).
* ``backward_error``: the normwise backward error of Rigal and Gaches,
  ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) (Higham, Accuracy and
  Stability of Numerical Algorithms, Thm 7.1).
* ``pivot_prefix_match``: the pivots must agree on every step up to the first
  step whose pivot column is not separated (gap < tau).
* ``closed_form_ipiv``: pivots of A = Pi * D when D's pivot order is the
  identity (column dominance), from the row placement alone.

Pins (tests/test_oracle_pins.py): both measures are checked against values
worked by hand on small cases chosen so that another norm, another dimension
factor or another eps gives a different number, and against planted errors in
factors and solutions that they must reject.
"""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def perm_from_ipiv(ipiv, m: int) -> np.ndarray:
    p = np.arange(m)
    for k, v in enumerate(np.asarray(ipiv)):
        j = int(v) - 1
        if j != k:
            p[k], p[j] = p[j], p[k]
    return p


def unpack(LU: np.ndarray):
    """(L, U) from the in-place factors: L unit lower m x p, U upper p x n."""
    m, n = LU.shape
    p = min(m, n)
    L = np.tril(LU[:, :p], -1).astype(np.float64)
    L[np.arange(p), np.arange(p)] = 1.0
    U = np.triu(LU[:p, :]).astype(np.float64)
    return L, U


def scaled_residual(A: np.ndarray, LU: np.ndarray, ipiv, eps: float = U64) -> float:
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m == 0 or n == 0:
        return 0.0
    L, U = unpack(np.asarray(LU))
    PA = A[perm_from_ipiv(ipiv, m), :]
    R = PA - L @ U
    na = np.abs(A).sum(axis=0).max()
    if na == 0.0:
        return 0.0 if not np.any(R) else np.inf
    return float(np.abs(R).sum(axis=0).max() / (max(m, n) * eps * na))


def backward_error(A: np.ndarray, x: np.ndarray, b: np.ndarray) -> float:
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = b - A @ x
    den = np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
    return float(np.abs(r).max() / den) if den > 0 else 0.0


def separated_prefix(gap, tau: float) -> int:
    """Number of leading steps whose pivot column is separated (gap >= tau)."""
    g = np.asarray(gap)
    bad = np.nonzero(g < tau)[0]
    return int(bad[0]) if len(bad) else len(g)


def pivot_prefix_match(ipiv_test, ipiv_ref, gap, tau: float = 1e-9):
    """(ok, n_compared, first_mismatch) over the separated prefix."""
    k = separated_prefix(gap, tau)
    a = np.asarray(ipiv_test)[:k]
    b = np.asarray(ipiv_ref)[:k]
    bad = np.nonzero(a != b)[0]
    return (len(bad) == 0, k, int(bad[0]) if len(bad) else -1)


def closed_form_ipiv(perm) -> np.ndarray:
    """Row perm[d] of A holds row d of a matrix whose partial-pivoting order is
    the identity; return the interchange vector partial pivoting produces on A."""
    perm = np.asarray(perm)
    m = len(perm)
    where = np.array(perm, copy=True)          # where[d] = current row of D-row d
    content = np.empty(m, dtype=np.int64)      # content[r] = D-row now at row r
    content[perm] = np.arange(m)
    ipiv = np.empty(m, dtype=np.int32)
    for k in range(m):
        r = where[k]
        ipiv[k] = r + 1
        if r != k:
            dk = content[k]
            content[k], content[r] = k, dk
            where[k], where[dk] = k, r
    return ipiv
