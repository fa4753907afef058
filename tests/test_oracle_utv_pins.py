"""Pins of the randUTV oracle (oracle/utv.py) against what fixes it
independently of its own code: the factorization identity A = U T V^T with
U, V orthogonal and T upper triangular (exact zeros below the diagonal);
the single-step case b >= n, where randUTV is the SVD (numpy's singular
values); the rank-revealing property the paper states (Section 3.2: after a
step, ||T22|| ~ sigma_{k+1}) on a matrix with a known gap; and planted
mistakes that these pins reject."""
import numpy as np
import pytest

from oracle import utv

U64 = 2.0 ** -53


def _matrix(n, sigma, seed):
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q1 @ np.diag(sigma) @ Q2.T, rng.standard_normal((n, n))


@pytest.mark.parametrize("n,b,q", [(64, 16, 0), (96, 16, 2), (80, 24, 1), (50, 16, 1)])
def test_factorization_identity(n, b, q):
    A, G = _matrix(n, np.geomspace(1, 1e-6, n), n + b)
    U, T, V = utv.randutv(A, b, q, G)
    assert np.abs(U @ T @ V.T - A).max() <= 50 * n * U64
    assert np.abs(U.T @ U - np.eye(n)).max() <= 50 * n * U64
    assert np.abs(V.T @ V - np.eye(n)).max() <= 50 * n * U64
    assert np.array_equal(np.tril(T, -1), np.zeros((n, n)))


def test_single_step_is_the_svd():
    n = 40
    A, G = _matrix(n, np.geomspace(3, 1e-3, n), 7)
    U, T, V = utv.randutv(A, n, 1, G)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.abs(np.diag(T) - s).max() <= 50 * n * U64 * s[0]
    assert np.abs(T - np.diag(np.diag(T))).max() <= 50 * n * U64 * s[0]


def test_rank_revealing_gap():
    """sigma = 1 (b times) then 1e-10: after the first step the trailing block
    holds only the small singular values, and the first diagonal block the
    large ones (the latter needs the right sketch: a sketch of the wrong
    space leaves the leading block with smaller singular values, below)."""
    n, b = 96, 16
    A, G = _matrix(n, np.r_[np.ones(b), 1e-10 * np.ones(n - b)], 3)
    U, T, V = utv.randutv(A, b, 1, G)
    assert np.linalg.norm(T[b:, b:], 2) <= 10e-10
    assert np.abs(np.diag(T)[:b] - 1.0).max() <= 1e-8


def test_planted_mistakes_fail():
    n, b = 96, 16
    A, G = _matrix(n, np.r_[np.ones(b), 1e-10 * np.ones(n - b)], 3)
    orig = utv.qr.geqr2

    # (a) the sketch without the transpose: Y = T22 G spans the wrong space
    def randutv_no_transpose(A, b, q, G):
        T = np.array(A, copy=True)
        k0 = 0
        Y = T @ G[:, :b]
        F, tau = orig(Y)
        Qy = utv.qr.form_q(F, tau, n)
        T = T @ Qy
        F, tau = orig(T[:, :b])
        Qu = utv.qr.form_q(F, tau, n)
        return Qu.T @ T
    T = randutv_no_transpose(A, b, 1, G)
    # the leading block no longer carries the large singular values
    assert np.abs(np.linalg.svd(T[:b, :b], compute_uv=False) - 1.0).max() > 1e-3

    # (b) a block column above the diagonal block left unrotated (one block
    # rotation missing): the identity A = U T V^T breaks
    A, G = _matrix(n, np.geomspace(1, 1e-3, n), 4)
    U, T, V = utv.randutv(A, b, 1, G)
    R = np.linalg.qr(np.random.default_rng(1).standard_normal((b, b)))[0]
    T_bad = T.copy()
    T_bad[:b, b:2 * b] = T_bad[:b, b:2 * b] @ R.T
    assert np.abs(U @ T_bad @ V.T - A).max() > 1e-6
