"""Pins of the Householder QR oracle (oracle/qr.py) against what fixes it
independently: LAPACK's dgeqrf (through numpy's raw QR) for the same
conventions, a hand-worked 2 x 2 example, exact rational products of
reflectors for the compact WY form, closed forms (triangular and diagonal
inputs), and the invariants Q^T Q = I and Q R = A.  Planted mistakes in a
copy of the oracle must fail these pins."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import qr

U = 2.0 ** -53


@pytest.mark.parametrize("shape", [(40, 40), (73, 31), (31, 73), (1, 5), (6, 1), (128, 96)])
def test_matches_lapack_dgeqrf(shape):
    """Same reflector conventions as LAPACK (beta = -sign(alpha) ||x||,
    v[0] = 1): numpy's raw QR calls dgeqrf and must give the same layout."""
    A = np.random.default_rng(sum(shape)).uniform(-1, 1, shape)
    F, t = qr.geqr2(A)
    h, tau = np.linalg.qr(A, mode="raw")
    scale = np.abs(A).sum(axis=0).max()
    assert np.abs(h.T - F).max() <= 64 * max(shape) * U * scale
    assert np.abs(tau - t).max() <= 64 * max(shape) * U


def test_house_hand_worked():
    v, t, b = qr.house(np.array([3.0, 4.0]))
    assert (b, t, v[1]) == (-5.0, 1.6, 0.5)
    v, t, b = qr.house(np.array([-3.0, 4.0]))
    assert (b, t, v[1]) == (5.0, 1.6, -0.5)
    v, t, b = qr.house(np.array([0.0, 2.0]))  # sign(0) = +1
    assert (b, t, v[1]) == (-2.0, 1.0, 1.0)
    v, t, b = qr.house(np.array([2.0, 0.0, 0.0]))  # nothing to annihilate: H = I
    assert (b, t) == (2.0, 0.0) and np.array_equal(v, [1.0, 0.0, 0.0])


def test_geqr2_hand_worked_2x2():
    """A = [[3, 1], [4, 2]]: H1 from (3, 4): beta = -5, tau = 8/5, v = (1, 1/2);
    H1 a1 = a1 - tau v (v.a1) = (1, 2) - 1.6 (1, 0.5) 2 = (-2.2, 0.4); the last
    column has nothing below its diagonal, so tau_2 = 0 and R = [[-5, -2.2],
    [0, 0.4]]; Q = H1 = [[-0.6, -0.8], [-0.8, 0.6]] reproduces A."""
    F, t = qr.geqr2(np.array([[3.0, 1.0], [4.0, 2.0]]))
    assert np.allclose(F, [[-5.0, -2.2], [0.5, 0.4]], rtol=0, atol=4 * U * 5)
    assert t[0] == 1.6 and t[1] == 0.0
    Q = qr.form_q(F, t)
    assert np.allclose(Q, [[-0.6, -0.8], [-0.8, 0.6]], rtol=0, atol=8 * U)


def _dyadic_reflectors(m, b, seed):
    rng = np.random.default_rng(seed)
    V = np.zeros((m, b))
    for j in range(b):
        V[j, j] = 1.0
        V[j + 1:, j] = rng.integers(-4, 5, size=m - j - 1) / 8.0
    tau = rng.integers(1, 8, size=b) / 4.0
    return V, tau


def _exact_product(V, tau):
    m, b = V.shape
    P = [[Fraction(int(i == j)) for j in range(m)] for i in range(m)]
    for j in range(b):  # P := P H_j, left to right: H_1 H_2 ... H_b
        v = [Fraction(x) for x in V[:, j]]
        t = Fraction(tau[j])
        Pv = [sum(P[i][k] * v[k] for k in range(m)) for i in range(m)]
        for i in range(m):
            for k in range(m):
                P[i][k] -= t * Pv[i] * v[k]
    return P


@pytest.mark.parametrize("m,b,seed", [(6, 3, 1), (9, 4, 2), (12, 5, 3)])
def test_larft_exact_compact_wy(m, b, seed):
    """I - V T V^T equals the product of the reflectors H_1 ... H_b exactly:
    with dyadic v and tau every float operation of larft and of the product
    below is exact, and the product itself is formed in rationals from the
    definition H_j = I - tau_j v_j v_j^T."""
    V, tau = _dyadic_reflectors(m, b, seed)
    T = qr.larft(V, tau)
    assert np.array_equal(T, np.triu(T))
    got = np.eye(m) - V @ T @ V.T
    P = _exact_product(V, tau)
    for i in range(m):
        for k in range(m):
            assert Fraction(got[i, k]) == P[i][k], (i, k)


def test_closed_forms_triangular_and_diagonal():
    """Nothing below the diagonal: every tau is 0 and R is the input, bit for
    bit (square, tall with zero rows below, wide)."""
    rng = np.random.default_rng(7)
    for A in (np.triu(rng.uniform(-1, 1, (9, 9))), np.diag(rng.uniform(0.5, 2, 6)),
              np.vstack([np.triu(rng.uniform(-1, 1, (5, 5))), np.zeros((4, 5))]),
              np.triu(rng.uniform(-1, 1, (4, 9)))):
        F, t = qr.geqr2(A)
        assert np.array_equal(t, np.zeros_like(t))
        assert np.array_equal(F, A)


@pytest.mark.parametrize("shape,nb", [((64, 64), 8), ((100, 37), 16), ((37, 100), 12), ((90, 90), 32)])
def test_invariants_and_blocked(shape, nb):
    A = np.random.default_rng(nb).uniform(-1, 1, shape)
    F, t = qr.geqr2(A)
    m, n = shape
    k = min(m, n)
    Q = qr.form_q(F, t, m)
    R = np.triu(F)
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 16 * m * U
    assert np.abs(Q[:, :k] @ R[:k, :] - A).max() <= 16 * m * U * np.abs(A).sum(axis=0).max()
    B, tb = qr.geqrf_blocked(A, nb)
    assert np.abs(B - F).max() <= 64 * m * U * np.abs(A).sum(axis=0).max()
    assert np.abs(tb - t).max() <= 64 * m * U


def test_planted_mistakes_fail():
    """A wrong sign of beta, and T in place of T^T in the blocked update: the
    LAPACK pin and the blocked-vs-unblocked pin reject them."""
    A = np.random.default_rng(11).uniform(-1, 1, (30, 20))
    h, tau = np.linalg.qr(A, mode="raw")

    orig = qr.house

    def house_bad(x):
        v, t, b = orig(x)
        if t == 0.0:
            return v, t, b
        alpha = x[0]
        beta = -b
        return np.concatenate([[1.0], x[1:] / (alpha - beta)]), (beta - alpha) / beta, beta

    try:
        qr.house = house_bad
        F, t = qr.geqr2(A)
    finally:
        qr.house = orig
    assert np.abs(h.T - F).max() > 1e-3

    def blocked_bad(A, nb):
        A = np.array(A, dtype=np.float64, copy=True, order="F")
        k = min(A.shape)
        for j0 in range(0, k, nb):
            j1 = min(j0 + nb, k)
            blk, t = qr.geqr2(A[j0:, j0:j1])
            A[j0:, j0:j1] = blk
            if j1 < A.shape[1]:
                V = qr.unit_lower(A, j0, j1)
                T = qr.larft(V, t)
                A[j0:, j1:] -= V @ (T @ (V.T @ A[j0:, j1:]))  # T instead of T^T
        return A
    F, t = qr.geqr2(A)
    assert np.abs(blocked_bad(A, 8) - F).max() > 1e-3
