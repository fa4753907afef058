"""CPU oracle for the Householder QR factorization -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the HIP path.

What it computes (the paper's HQR, Section 2.2: an upper triangular R, a unit
lower triangular V holding the Householder vectors and a vector of their
scalars; the compact WY form of a product of reflectors, Section 2.3):

* ``house(x)``: the reflector H = I - tau v v^T with v[0] = 1 that maps x to
  beta e_1 (Golub & Van Loan, Section 5.1.2, with LAPACK's choice of sign):
  alpha = x[0], s = ||x[1:]||_2; if s == 0: tau = 0, beta = alpha (H = I);
  else beta = -sign(alpha) sqrt(alpha^2 + s^2), tau = (beta - alpha) / beta,
  v[1:] = x[1:] / (alpha - beta).  sign(0) = +1.
* ``geqr2(A)``: unblocked HQR, one column at a time (k = min(m, n) steps):
  the reflector of A[j:, j], R[j, j] = beta, v[1:] stored below the diagonal,
  then A[j:, j+1:] := H A[j:, j+1:] as w = v^T A[j:, j+1:], A -= tau v w.
  Output in LAPACK geqrf's layout: R on and above the diagonal, V strictly
  below it (unit diagonal implied), tau.
* ``larft(V, tau)``: T upper triangular with Q = H_1 H_2 ... H_b = I - V T V^T
  (the compact WY form, Schreiber & Van Loan): T[j, j] = tau_j,
  T[:j, j] = -tau_j T[:j, :j] V[:, :j]^T v_j.
* ``geqrf_blocked(A, nb)``: the blocked right-looking form: per block of nb
  columns, geqr2 of the block column, T = larft, and the trailing columns
  A2 := Q^T A2 = A2 - V (T^T (V^T A2)).  Equal to geqr2 up to rounding.
* ``form_q(QR, tau)``: Q = H_1 ... H_k applied to the identity's first
  columns (for the checks).

The paper writes the product of b reflectors as I - W T W^* with T upper
triangular without fixing the order of the factors; this module takes
Q = H_1 ... H_b = I - V T V^T (T upper triangular), so that the update of the
trailing columns, Q^T A2, uses T^T.

The sums of squares are formed plainly (no scaling against overflow): inputs
whose squares overflow are outside what is checked.
"""
from __future__ import annotations

import math

import numpy as np


def house(x: np.ndarray):
    """(v, tau, beta) of the reflector that maps x to beta e_1."""
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    s2 = float(np.dot(x[1:], x[1:]))
    v = np.zeros_like(x)
    v[0] = 1.0
    if s2 == 0.0:
        return v, 0.0, alpha
    beta = -math.copysign(math.sqrt(alpha * alpha + s2), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def geqr2(A: np.ndarray):
    """Unblocked HQR; returns (QR in geqrf's layout, tau)."""
    A = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = A.shape
    k = min(m, n)
    tau = np.zeros(k)
    for j in range(k):
        v, t, beta = house(A[j:, j])
        tau[j] = t
        A[j, j] = beta
        A[j + 1:, j] = v[1:]
        if j + 1 < n and t != 0.0:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= t * np.outer(v, w)
    return A, tau


def unit_lower(QR: np.ndarray, j0: int, j1: int) -> np.ndarray:
    """The explicit V (rows j0.., columns j0..j1-1) with its unit diagonal and
    zeros above it."""
    V = np.tril(QR[j0:, j0:j1], -1)
    V[np.arange(j1 - j0), np.arange(j1 - j0)] = 1.0
    return V


def larft(V: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """T of the compact WY form H_1 ... H_b = I - V T V^T."""
    b = len(tau)
    T = np.zeros((b, b))
    for j in range(b):
        T[j, j] = tau[j]
        if j:
            T[:j, j] = -tau[j] * (T[:j, :j] @ (V[:, :j].T @ V[:, j]))
    return T


def geqrf_blocked(A: np.ndarray, nb: int):
    """Blocked right-looking HQR with compact WY updates; (QR, tau)."""
    A = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = A.shape
    k = min(m, n)
    tau = np.zeros(k)
    for j0 in range(0, k, nb):
        j1 = min(j0 + nb, k)
        blk, t = geqr2(A[j0:, j0:j1])
        A[j0:, j0:j1] = blk
        tau[j0:j1] = t
        if j1 < n:
            V = unit_lower(A, j0, j1)
            T = larft(V, t)
            A2 = A[j0:, j1:]
            A[j0:, j1:] = A2 - V @ (T.T @ (V.T @ A2))
    return A, tau


def form_q(QR: np.ndarray, tau: np.ndarray, ncols: int | None = None) -> np.ndarray:
    """The first ncols columns of Q = H_1 ... H_k (default k)."""
    m = QR.shape[0]
    k = len(tau)
    ncols = k if ncols is None else ncols
    Q = np.eye(m, ncols)
    for j in reversed(range(k)):
        v = np.zeros(m)
        v[j] = 1.0
        v[j + 1:] = QR[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q


def r_factor(QR: np.ndarray) -> np.ndarray:
    k = min(QR.shape)
    return np.triu(QR[:k, :])
