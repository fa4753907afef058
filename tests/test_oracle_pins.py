"""Pins of the CPU oracle against facts fixed by mathematics, not by the oracle.

Every check here would fail on a plausible mistake in the oracle (wrong tie
break, missing interchange of the left columns, transposed update, reciprocal
instead of division, dropped update term, wrong ipiv base):

* brute force over all row orderings in exact rational arithmetic (n = 4..8):
  with unique column maxima exactly one permutation gives |L| <= 1;
* exact stepwise elimination and the loop invariant in rationals (n = 9..16);
* the floating-point loop invariant after every step, elementwise within the
  standard backward-error bound gamma_k |L||U|;
* closed forms: identity, permutation matrices, triangular matrices, Pi*D with
  column dominance, exactly factorable dyadic matrices (bit-exact L and U);
* a hand-worked example (tests/golden/lupp_4x4_worked.txt);
* LAPACK's dgetrf through scipy (run only) on separated inputs;
* right- vs left-looking and 1 vs N threads: bitwise identical.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import checks

pytestmark = pytest.mark.usefixtures("oracle_lib")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oracle():
    import oracle
    return oracle


# ---------------------------------------------------------------- exact helpers
def _exact_nopivot_lu(rows):
    """Exact unpivoted LU of a list of Fraction rows; None if a zero pivot or a
    multiplier of magnitude > 1 appears (such a row order cannot be partial
    pivoting's)."""
    S = [list(r) for r in rows]
    n = len(S)
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for k in range(n):
        piv = S[k][k]
        if piv == 0:
            return None
        for i in range(k + 1, n):
            l = S[i][k] / piv
            if abs(l) > 1:
                return None
            L[i][k] = l
            for j in range(k, n):
                S[i][j] -= l * S[k][j]
    return L, S


def _valid_orders_dfs(A):
    """All row orders whose unpivoted LU has |L| <= 1 (exhaustive search over
    orderings; a prefix with a multiplier > 1 cannot extend to a valid one)."""
    n = len(A)
    out = []

    def rec(order, S):
        k = len(order)
        if k == n:
            out.append(tuple(order))
            return
        # S: dict row-> current (Schur) row for unused rows
        for r in list(S.keys()):
            piv = S[r][k]
            if piv == 0:
                continue
            ok = all(abs(S[q][k]) <= abs(piv) for q in S if q != r)
            if not ok:
                continue
            T = {}
            for q in S:
                if q == r:
                    continue
                l = S[q][k] / piv
                T[q] = [S[q][j] - l * S[r][j] for j in range(n)]
            rec(order + [r], T)

    rec([], {i: [Fraction(int(x)) for x in A[i]] for i in range(n)})
    return out


def _exact_lupp(A):
    """Exact rational partial pivoting (lowest index among exact maxima).
    Returns (perm, L, U, states) with states[k] = (perm_k, L_k, S_k) for the
    invariant check."""
    n = len(A)
    M = [[Fraction(int(x)) for x in row] for row in A]
    perm = list(range(n))
    for k in range(n):
        col = [abs(M[i][k]) for i in range(k, n)]
        best = max(col)
        piv = k + col.index(best)
        if piv != k:
            M[k], M[piv] = M[piv], M[k]
            perm[k], perm[piv] = perm[piv], perm[k]
        if M[k][k] == 0:
            continue
        for i in range(k + 1, n):
            M[i][k] = M[i][k] / M[k][k]
            for j in range(k + 1, n):
                M[i][j] -= M[i][k] * M[k][j]
    return perm, M


def _int_matrix(seed, n, lo=-9, hi=9):
    return synth.stream(seed, 77).integers(lo, hi + 1, size=(n, n)).astype(np.float64)


def _exact_unique_maxima(A):
    """True when exact partial pivoting never meets a tie for the maximum."""
    n = len(A)
    M = [[Fraction(int(x)) for x in row] for row in A]
    for k in range(n):
        col = [abs(M[i][k]) for i in range(k, n)]
        best = max(col)
        if best == 0 or col.count(best) > 1:
            return False
        piv = k + col.index(best)
        M[k], M[piv] = M[piv], M[k]
        for i in range(k + 1, n):
            l = M[i][k] / M[k][k]
            for j in range(k, n):
                M[i][j] -= l * M[k][j]
    return True


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_bruteforce_pivot_order(n):
    o = _oracle()
    done = 0
    seed = 1000 * n
    while done < (3 if n <= 6 else 1):
        seed += 1
        A = _int_matrix(seed, n)
        if not _exact_unique_maxima(A):
            continue
        if n <= 6:  # full enumeration of all n! orderings
            valid = []
            for order in itertools.permutations(range(n)):
                if _exact_nopivot_lu([[Fraction(int(x)) for x in A[i]] for i in order]) is not None:
                    valid.append(order)
        else:
            valid = _valid_orders_dfs(A)
        assert len(valid) == 1, valid
        LU, ipiv, info = o.getrf(A)
        assert info == 0
        p = checks.perm_from_ipiv(ipiv, n)
        assert tuple(int(x) for x in p) == valid[0]
        # factors agree with the exact ones to rounding
        Lx, Ux = _exact_nopivot_lu([[Fraction(int(x)) for x in A[i]] for i in valid[0]])
        Lf = np.array([[float(v) for v in r] for r in Lx])
        Uf = np.triu(np.array([[float(v) for v in r] for r in Ux]))
        L, U = checks.unpack(LU)
        scale = np.abs(A).max() * n
        assert np.abs(L - Lf).max() <= 1e-12 * n
        assert np.abs(U - Uf).max() <= 1e-12 * scale
        done += 1


@pytest.mark.parametrize("n", [9, 12, 16])
def test_exact_stepwise_and_invariant(n):
    o = _oracle()
    seed = 7000 + n
    while True:
        seed += 1
        A = _int_matrix(seed, n, -5, 5)
        if _exact_unique_maxima(A):
            break
    perm, M = _exact_lupp(A)
    # exact invariant at the end: P A == L U in rationals
    L = [[(M[i][j] if j < i else Fraction(int(i == j))) for j in range(n)] for i in range(n)]
    U = [[(M[i][j] if j >= i else Fraction(0)) for j in range(n)] for i in range(n)]
    for i in range(n):
        for j in range(n):
            assert sum(L[i][k] * U[k][j] for k in range(n)) == int(A[perm[i]][j])
    LU, ipiv, info = o.getrf(A)
    assert [int(x) for x in checks.perm_from_ipiv(ipiv, n)] == perm
    Lf = np.array([[float(v) for v in r] for r in L])
    assert np.abs(np.tril(LU, -1) - np.tril(Lf, -1)).max() <= 1e-12 * n


# ---------------------------------------------------------------- FP64 invariant
@pytest.mark.parametrize("shape", [(5, 5), (9, 9), (16, 16), (12, 7), (7, 12), (1, 6), (6, 1)])
def test_loop_invariant_every_step(shape):
    o = _oracle()
    m, n = shape
    A = synth.uniform(11, 3, m, n)
    p = min(m, n)
    u = checks.U64
    for k in range(p + 1):
        M, ipiv, info = o.getrf(A, ksteps=k)
        assert info == 0
        Lf = np.eye(m)
        Lf[:, :k] = np.tril(M[:, :k], -1) + np.eye(m)[:, :k]
        Uf = np.zeros((m, n))
        Uf[:k, :] = np.triu(M[:k, :])
        Uf[k:, k:] = M[k:, k:]
        PA = A[checks.perm_from_ipiv(ipiv, m), :]
        R = np.abs(PA - Lf @ Uf)
        gam = (k + 1) * u / (1 - (k + 1) * u)
        bound = gam * (np.abs(Lf) @ np.abs(Uf)) + 1e-300
        assert np.all(R <= bound), (k, float((R / bound).max()))
        assert np.abs(M[:, :k][np.tril_indices(m, -1, k)]).max(initial=0.0) <= 1.0


def test_invariant_catches_planted_mistake():
    """The invariant check rejects an elimination with one dropped term."""
    A = synth.uniform(12, 3, 8, 8)
    o = _oracle()
    M, ipiv, _ = o.getrf(A, ksteps=3)
    M[5, 6] += 0.1  # plant: a missing update term
    Lf = np.eye(8)
    Lf[:, :3] = np.tril(M[:, :3], -1) + np.eye(8)[:, :3]
    Uf = np.zeros((8, 8))
    Uf[:3, :] = np.triu(M[:3, :])
    Uf[3:, 3:] = M[3:, 3:]
    PA = A[checks.perm_from_ipiv(ipiv, 8), :]
    gam = 4 * checks.U64
    assert not np.all(np.abs(PA - Lf @ Uf) <= gam * (np.abs(Lf) @ np.abs(Uf)))


# ---------------------------------------------------------------- closed forms
def test_identity():
    o = _oracle()
    LU, ipiv, info = o.getrf(np.eye(37))
    assert info == 0 and np.array_equal(ipiv, np.arange(1, 38)) and np.array_equal(LU, np.eye(37))


@pytest.mark.parametrize("n", [2, 17, 64])
def test_permutation_matrix(n):
    o = _oracle()
    perm = synth.permutation(5, 9, n)
    A = np.zeros((n, n), order="F")
    A[perm, np.arange(n)] = 1.0  # row perm[i] holds e_i^T
    LU, ipiv, info = o.getrf(A)
    assert info == 0
    assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))
    assert np.array_equal(LU, np.eye(n))


def test_upper_triangular_bit_exact():
    o = _oracle()
    A = np.triu(synth.uniform(3, 4, 40, 40)) + 3.0 * np.eye(40)
    LU, ipiv, info = o.getrf(A)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, 41)) and np.array_equal(LU, A)


@pytest.mark.parametrize("n", [50, 300])
def test_pi_times_column_dominant(n):
    o = _oracle()
    A, perm = synth.pi_times_coldom(21, 4, n)
    LU, ipiv, info = o.getrf(A)
    assert info == 0
    assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))
    assert checks.scaled_residual(A, LU, ipiv) < 10


@pytest.mark.parametrize("n", [1, 2, 64, 257])
def test_exactly_factorable_bit_exact(n):
    o = _oracle()
    A, L, U, perm = synth.exact_lu_product(8, 30, n)
    LU, ipiv, info = o.getrf(A)
    assert info == 0
    assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))
    Lo, Uo = checks.unpack(LU)
    assert np.array_equal(Lo, L) and np.array_equal(Uo, U)
    LU32, ipiv32, info32 = o.getrf(A.astype(np.float32))
    assert np.array_equal(ipiv32, ipiv) and np.array_equal(LU32.astype(np.float64), LU)


def test_tie_break_lowest_index():
    o = _oracle()
    A = np.array([[2.0, 1, 0], [-2.0, 5, 1], [1.0, 0, 4]], order="F")
    _, ipiv, _ = o.getrf(A)
    assert ipiv[0] == 1
    B = np.array([[1.0, 1, 0], [-2.0, 5, 1], [2.0, 0, 4]], order="F")
    _, ipiv, _ = o.getrf(B)
    assert ipiv[0] == 2


def test_golden_worked_example():
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "lupp_4x4_worked.txt"))
             if ln.strip() and not ln.startswith("#")]
    sec = {}
    cur = None
    for ln in lines:
        if ln in ("A", "IPIV", "L", "U"):
            cur = ln
            sec[cur] = []
        else:
            sec[cur].append([Fraction(t) for t in ln.split()])
    A = np.array([[float(v) for v in r] for r in sec["A"]], order="F")
    LU, ipiv, info = _oracle().getrf(A)
    assert info == 0 and [int(x) for x in ipiv] == [int(v) for v in sec["IPIV"][0]]
    L, U = checks.unpack(LU)
    assert np.allclose(L, np.array([[float(v) for v in r] for r in sec["L"]]), rtol=0, atol=4e-16)
    assert np.allclose(U, np.array([[float(v) for v in r] for r in sec["U"]]), rtol=0, atol=4e-15)


# ---------------------------------------------------------------- singular
def test_zero_column_info():
    o = _oracle()
    A = synth.uniform(4, 1, 10, 10)
    A[:, 6] = 0.0
    A[:, 7] = A[:, 7] * 0  # two zero columns: info reports the first
    LU, ipiv, info = o.getrf(A)
    assert info == 7


def test_zero_matrix():
    LU, ipiv, info = _oracle().getrf(np.zeros((5, 5)))
    assert info == 1 and np.array_equal(ipiv, np.arange(1, 6))


# ---------------------------------------------------------------- properties
@pytest.mark.parametrize("shape", [(512, 512), (300, 200), (200, 300), (1, 1), (64, 1)])
def test_l_bounded_ipiv_range_residual(shape):
    o = _oracle()
    m, n = shape
    A = synth.uniform(20210512, 0, m, n)
    LU, ipiv, info = o.getrf(A)
    assert info == 0
    L, U = checks.unpack(LU)
    assert np.abs(L).max() <= 1.0
    k = np.arange(len(ipiv))
    assert np.all(ipiv >= k + 1) and np.all(ipiv <= m)
    p = checks.perm_from_ipiv(ipiv, m)
    assert np.array_equal(np.sort(p), np.arange(m))
    P = np.eye(m)[p]
    assert np.array_equal(P @ P.T, np.eye(m))
    assert checks.scaled_residual(A, LU, ipiv) < 10


def test_scipy_lapack_agrees():
    import scipy.linalg as sl
    o = _oracle()
    for n in (64, 512):
        A = synth.uniform(5, 2, n, n)
        LU, ipiv, info, gap = o.getrf(A, with_gap=True)
        lu2, piv2 = sl.lu_factor(A)
        ok, cmp, first = checks.pivot_prefix_match(piv2 + 1, ipiv, gap, 1e-9)
        assert ok and cmp == n, (cmp, first)
        assert checks.scaled_residual(A, LU, ipiv) < 10
        assert checks.scaled_residual(A, lu2, piv2 + 1) < 10


def test_left_looking_bitwise():
    o = _oracle()
    for (m, n) in [(64, 64), (150, 100), (100, 150)]:
        A = synth.uniform(9, 8, m, n)
        a1, p1, i1 = o.getrf(A)
        a2, p2, i2 = o.getrf_left(A)
        assert i1 == i2 and np.array_equal(p1, p2) and np.array_equal(a1.view(np.int64), a2.view(np.int64))


def test_threads_bitwise():
    o = _oracle()
    A = synth.uniform(9, 9, 400, 400)
    a1, p1, _ = o.getrf(A, nthreads=1)
    a2, p2, _ = o.getrf(A, nthreads=4)
    assert np.array_equal(p1, p2) and np.array_equal(a1.view(np.int64), a2.view(np.int64))


def test_getrs_solution():
    o = _oracle()
    for n in (1, 7, 200):
        A = synth.uniform(31, 0, n, n)
        b = synth.uniform(31, 1, n, 1)[:, 0]
        LU, ipiv, info = o.getrf(A)
        x, st = o.getrs(LU, ipiv, b)
        assert st == 0
        assert checks.backward_error(A, x, b) < 4 * n * checks.U64
        xr = np.linalg.solve(A, b)
        kappa = np.linalg.cond(A, 1)
        assert np.abs(x - xr).max() / np.abs(xr).max() < 10 * n * kappa * checks.U64


def test_getrs_refuses_singular():
    o = _oracle()
    A = synth.uniform(4, 1, 6, 6)
    A[:, 2] = 0.0
    LU, ipiv, info = o.getrf(A)
    _, st = o.getrs(LU, ipiv, np.ones(6))
    assert info == 3 and st == 3


def test_fp32_oracle():
    o = _oracle()
    A = synth.uniform(40, 0, 300, 300)
    LU, ipiv, info, gap = o.getrf(A.astype(np.float32), with_gap=True)
    assert info == 0 and LU.dtype == np.float32
    assert checks.scaled_residual(A.astype(np.float32), LU, ipiv, checks.U32) < 10
    _, ipiv64, _, gap64 = o.getrf(A, with_gap=True)
    ok, k, first = checks.pivot_prefix_match(ipiv, ipiv64, gap64, 1e-4)
    assert ok, (k, first)


def test_batched_oracle_matches_single():
    o = _oracle()
    sizes = synth.batch_sizes(3, 40, 1, 30)
    A, aoff, B, boff = synth.batch_uniform(3, sizes)
    LU, ipiv, poff, X, info = o.gesv_batched(sizes, A, aoff, B, boff, nthreads=4)
    assert np.all(info == 0)
    for s in (0, 7, 39):
        n = int(sizes[s])
        As = A[aoff[s]:aoff[s] + n * n].reshape(n, n, order="F")
        l1, p1, _ = o.getrf(As)
        assert np.array_equal(l1.ravel(order="F"), LU[aoff[s]:aoff[s] + n * n])
        assert np.array_equal(p1, ipiv[poff[s]:poff[s] + n])
        x1, _ = o.getrs(l1, p1, B[boff[s]:boff[s] + n])
        assert np.array_equal(x1, X[boff[s]:boff[s] + n])


def test_closed_form_ipiv_helper_small():
    # hand-checked: rows holding D-rows (0,1,2) at (2,0,1)
    assert list(checks.closed_form_ipiv([2, 0, 1])) == [3, 3, 3]
    assert list(checks.closed_form_ipiv([0, 1, 2])) == [1, 2, 3]
    assert list(checks.closed_form_ipiv([1, 0, 2])) == [2, 2, 3]


def test_synth_fast_generator_matches_numpy_philox():
    """The threaded C fill reproduces numpy's Philox-4x64-10 stream exactly."""
    for (m, n, lo, hi) in [(1, 1, -1.0, 1.0), (7, 5, -1.0, 1.0), (33, 17, -0.5, 0.5), (64, 3, 0.0, 1.0)]:
        a = synth.uniform(123, 9, m, n, lo, hi)
        b = synth.uniform_numpy(123, 9, m, n, lo, hi)
        assert a.flags["F_CONTIGUOUS"] and np.array_equal(a, b)


# ---------------------------------------------------------------- acceptance measures
# The two numbers every parity test checks against its bound are pinned here by
# hand-worked values.  Each case is built so that the plausible slips give a
# different number: the infinity norm in place of the 1-norm, n^2 or min(m,n) in
# place of max(m,n), eps = 1 or DBL_EPSILON in place of the unit roundoff, an
# unpermuted A, or the 1-norm of r, x or b in the backward error.

def test_scaled_residual_hand_worked():
    # A is upper triangular: P = I, L = I, U = A.  ||A||_1 = 2 (column sums
    # 1, 2, 2), ||A||_inf = 3.  Planting delta at L(1,0) adds delta * U(0,:) =
    # delta * (1, 1, 1) to row 1 of L*U (exact in binary64 for delta = 30u), so
    # ||PA - LU||_1 = delta and ||PA - LU||_inf = 3 delta.
    u = checks.U64
    A = np.array([[1.0, 1, 1], [0, 1, 0], [0, 0, 1]], order="F")
    LU = A.copy(order="F")
    delta = 30 * u
    LU[1, 0] = delta
    ipiv = np.array([1, 2, 3], dtype=np.int32)
    # delta / (max(m,n) * u * ||A||_1) = 30u / (3 * u * 2) = 5 exactly
    assert checks.scaled_residual(A, LU, ipiv) == 5.0
    # the same planted error measured against FP32's unit roundoff
    assert checks.scaled_residual(A, LU, ipiv, checks.U32) == 30 * u / (3 * checks.U32 * 2)
    # an exact factorization scores 0
    assert checks.scaled_residual(A, A, ipiv) == 0.0


def test_scaled_residual_uses_max_dimension_and_permutation():
    # 4 x 2, A = P^T * [I; 0] with rows swapped: ipiv (2, 2) swaps rows 0 and 1.
    u = checks.U64
    A = np.array([[0.0, 1], [1, 0], [0, 0], [0, 0]], order="F")
    LU = np.array([[1.0, 0], [0, 1], [0, 0], [0, 0]], order="F")
    ipiv = np.array([2, 2], dtype=np.int32)
    assert checks.scaled_residual(A, LU, ipiv) == 0.0
    # the unpermuted comparison would see ||A - LU||_1 = 2
    assert checks.scaled_residual(A, LU, np.array([1, 2], dtype=np.int32)) == 2.0 / (4 * u * 1.0)
    # planted error 8u at L(3,1): ||R||_1 = 8u, max(m,n) = 4, ||A||_1 = 1 -> 2
    LU[3, 1] = 8 * u
    assert checks.scaled_residual(A, LU, ipiv) == 2.0


def test_scaled_residual_rejects_perturbed_factors():
    o = _oracle()
    A = synth.uniform(77, 5, 60, 60)
    LU, ipiv, info = o.getrf(A)
    assert checks.scaled_residual(A, LU, ipiv) < 10
    bad = LU.copy(order="F")
    bad[40, 7] += 1e-9  # one wrong multiplier
    assert checks.scaled_residual(A, bad, ipiv) > 1e3
    bad = LU.copy(order="F")
    bad[7, 40] *= 1 + 1e-10  # one wrong U entry
    assert checks.scaled_residual(A, bad, ipiv) > 10
    wrong = ipiv.copy()
    wrong[3], wrong[4] = wrong[4], wrong[3]
    if not np.array_equal(wrong, ipiv):
        assert checks.scaled_residual(A, LU, wrong) > 1e3


def test_backward_error_hand_worked():
    # A = [[1, 2], [1, 0]]: ||A||_inf = 3 (row sums 3, 1), ||A||_1 = 2.
    # x = (1, -2): A x = (-3, 1).  b = (-2.5, 2): r = b - A x = (0.5, 1),
    # ||r||_inf = 1, ||x||_inf = 2, ||b||_inf = 2.5.
    # eta = 1 / (3 * 2 + 2.5) = 2/17 (any other norm gives another value).
    A = np.array([[1.0, 2], [1, 0]], order="F")
    x = np.array([1.0, -2])
    b = np.array([-2.5, 2.0])
    assert checks.backward_error(A, x, b) == 1.0 / 8.5
    # the exact solution has eta = 0
    xs = np.linalg.solve(A, b)
    assert checks.backward_error(A, xs, b) <= 2 * checks.U64
    # zero data: defined as 0
    assert checks.backward_error(np.zeros((2, 2)), np.zeros(2), np.zeros(2)) == 0.0


def test_backward_error_rejects_perturbed_solution():
    o = _oracle()
    n = 80
    A = synth.uniform(78, 0, n, n)
    b = synth.uniform(78, 1, n, 1)[:, 0]
    LU, ipiv, _ = o.getrf(A)
    x, st = o.getrs(LU, ipiv, b)
    assert checks.backward_error(A, x, b) <= 8 * n * checks.U64
    y = x.copy()
    y[17] += 1e-8 * np.abs(x).max()
    assert checks.backward_error(A, y, b) > 1e3 * n * checks.U64


def test_gap_hand_worked():
    """gap_k on the worked 4 x 4 example: column maxima 4 vs 4 (tie), then
    4 vs 1, then 11/4 vs 5/4, then a single row."""
    A = np.array([[1.0, 2, 0, 1], [4, 4, 2, 0], [2, 1, 3, 1], [-4, 0, 1, 2]], order="F")
    _, _, _, gap = _oracle().getrf(A, with_gap=True)
    assert gap[0] == 0.0
    assert gap[1] == 0.75
    assert gap[2] == (2.75 - 1.25) / 2.75
    assert gap[3] == 1.0
    assert checks.separated_prefix(gap, 1e-9) == 0
    assert checks.separated_prefix(np.array([0.5, 0.2, 1e-12, 1.0]), 1e-9) == 2


# ---------------------------------------------------------------- FP32 solve and batched driver
def _dyadic_system(seed, n, dtype):
    """A = Pi^T L U with exactly factorable dyadic factors and an integer x:
    b = A x, every partial sum of the solve is a multiple of 1/4 bounded by
    a few hundred, so a correct solve returns x exactly in binary32."""
    A, L, U, perm = synth.exact_lu_product(seed, 31, n)
    x = synth.stream(seed, 32).integers(-3, 4, size=n).astype(np.float64)
    b = A @ x
    return A.astype(dtype), b.astype(dtype), x


@pytest.mark.parametrize("n", [1, 5, 16, 40])
def test_sgetrs_exact_dyadic(n):
    o = _oracle()
    A, b, x = _dyadic_system(900 + n, n, np.float32)
    LU, ipiv, info = o.getrf(A)
    assert info == 0 and LU.dtype == np.float32
    xs, st = o.getrs(LU, ipiv, b)
    assert st == 0 and xs.dtype == np.float32
    assert np.array_equal(xs.astype(np.float64), x)
    # two right-hand sides at once, the second the negated first
    X, st = o.getrs(LU, ipiv, np.stack([b, -b], axis=1))
    assert st == 0 and np.array_equal(X[:, 0].astype(np.float64), x) and np.array_equal(X[:, 1].astype(np.float64), -x)


def test_sgetrs_refuses_singular_and_bounds_error():
    o = _oracle()
    A = synth.uniform(5, 1, 7, 7).astype(np.float32)
    A[:, 4] = 0
    LU, ipiv, info = o.getrf(A)
    _, st = o.getrs(LU, ipiv, np.ones(7, dtype=np.float32))
    assert info == 5 and st == 5
    n = 120
    A = synth.uniform(6, 1, n, n).astype(np.float32)
    b = synth.uniform(6, 2, n, 1)[:, 0].astype(np.float32)
    LU, ipiv, _ = o.getrf(A)
    x, _ = o.getrs(LU, ipiv, b)
    assert checks.backward_error(A, x, b) <= 8 * n * checks.U32


def test_batched_oracle_exact_dyadic_systems():
    """Every system of a packed batch of exactly factorable systems comes back
    with its exact pivots, factors and solution, in both precisions."""
    o = _oracle()
    sizes = np.array([1, 3, 8, 17, 2, 33], dtype=np.int32)
    for dtype in (np.float64, np.float32):
        blocks, rhs, sols, facs = [], [], [], []
        for i, n in enumerate(sizes):
            A, L, U, perm = synth.exact_lu_product(500 + i, 31, int(n))
            x = synth.stream(500 + i, 32).integers(-3, 4, size=int(n)).astype(np.float64)
            blocks.append(A.ravel(order="F"))
            rhs.append(A @ x)
            sols.append(x)
            facs.append((L, U, checks.closed_form_ipiv(perm)))
        a_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)[:-1]])
        b_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))[:-1]])
        Ap = np.concatenate(blocks).astype(dtype)
        Bp = np.concatenate(rhs).astype(dtype)
        LU, ipiv, p_off, X, info = o.gesv_batched(sizes, Ap, a_off, Bp, b_off, nthreads=3)
        assert np.all(info == 0) and LU.dtype == dtype and X.dtype == dtype
        for i, n in enumerate(sizes):
            n = int(n)
            L, U, ip = facs[i]
            Ls, Us = checks.unpack(LU[a_off[i]:a_off[i] + n * n].reshape(n, n, order="F"))
            assert np.array_equal(ipiv[p_off[i]:p_off[i] + n], ip)
            assert np.array_equal(Ls, L) and np.array_equal(Us, U)
            assert np.array_equal(X[b_off[i]:b_off[i] + n].astype(np.float64), sols[i])


def test_batched_oracle_zero_pivot_leaves_rhs():
    o = _oracle()
    sizes = np.array([4, 5], dtype=np.int32)
    A, aoff, B, boff = synth.batch_uniform(8, sizes)
    A[aoff[1] + 2 * 5:aoff[1] + 3 * 5] = 0.0  # column 2 of system 1 is zero
    LU, ipiv, poff, X, info = o.gesv_batched(sizes, A, aoff, B, boff, nthreads=2)
    assert info[0] == 0 and info[1] == 3
    assert np.array_equal(X[boff[1]:boff[1] + 5], B[boff[1]:boff[1] + 5])
    assert checks.backward_error(A[:16].reshape(4, 4, order="F"), X[:4], B[:4]) <= 32 * checks.U64
