/*
 * CPU oracle for LU factorization with partial pivoting (P*A = L*U).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP path.
 *
 * What it computes.  The paper states its problem for a dense real m x n
 * matrix with the submatrix notation A(c:d, e:f) (Preliminaries, Section 2),
 * keeps the factors in place of the input (Section 3.2: one matrix is stored
 * and overwritten at every step; Section 2.2: reflector data stored below the
 * diagonal), and builds its factorization right-looking, one block of columns
 * per step (Section 3.2).  It names the column-block ("panel") factorization
 * as the step that limits blocked LU (Section 4.1).  It does not spell out
 * LU itself; the definition used here is the textbook one (Golub & Van Loan,
 * cited by the paper) with the conventions of LAPACK's getf2:
 *
 *   for k = 0 .. min(m,n)-1:
 *     piv = the lowest row index i >= k with |a(i,k)| maximal
 *           (sequential scan, strict ">" comparison);
 *     ipiv[k] = piv + 1                               (1-based interchange)
 *     if a(piv,k) == 0: info = k+1 (first such k); nothing else this step
 *     else: swap rows k and piv across all n columns;
 *           a(i,k) = a(i,k) / a(k,k) for i > k         (true division)
 *           a(i,j) = a(i,j) - a(i,k)*a(k,j) for i,j > k
 *                     (product and difference rounded separately)
 *
 * This is the right-looking loop of the paper's FLAME notation (Section 4.3:
 * partition, repartition with a b x b diagonal block, continue-with) with
 * block size b = 1.  Each element (i,j) receives its updates in increasing k,
 * so the left-looking variant below and the threaded variant are bitwise
 * identical to the sequential right-looking one.  Build with
 * -ffp-contract=off and without fast-math so no fused multiply-add appears.
 *
 * Pins (tests/test_oracle_pins.py): brute-force enumeration of permutations
 * in exact rational arithmetic for orders 4..8, exact stepwise elimination for
 * orders 9..16, the loop invariant after every step, |L| <= 1, closed forms
 * (identity, permutation, triangular, Pi*D with column dominance, exactly
 * factorable dyadic matrices), LAPACK's dgetrf via scipy, and the scaled
 * residual.  The FP32 solve and the batched driver are pinned by exactly
 * factorable dyadic systems with integer solutions (pivots, factors and x
 * bit for bit, in both precisions) and by the per-system calls; the pivot
 * separation gap by a hand-worked example.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* gap_k = (|v1| - |v2|) / |v1| over the pivot column's top two magnitudes;
 * 1 when only one candidate row remains, 0 when the column is all zero. */
#define DEFINE_GETRF(T, NAME, FABS)                                                    \
  int NAME(int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, double* gap,        \
           int64_t ksteps, int nthreads) {                                             \
    int64_t p = m < n ? m : n;                                                         \
    int info = 0;                                                                      \
    if (ksteps >= 0 && ksteps < p) p = ksteps;                                         \
    (void)nthreads;                                                                    \
    for (int64_t k = 0; k < p; ++k) {                                                  \
      int64_t piv = k;                                                                 \
      T best = FABS(A[IDX(k, k, lda)]);                                                \
      T second = (T)-1;                                                                \
      for (int64_t i = k + 1; i < m; ++i) {                                            \
        T v = FABS(A[IDX(i, k, lda)]);                                                 \
        if (v > best) { second = best; best = v; piv = i; }                            \
        else if (v > second) { second = v; }                                           \
      }                                                                                \
      if (gap) {                                                                       \
        if (k + 1 >= m) gap[k] = 1.0;                                                  \
        else if (best == (T)0) gap[k] = 0.0;                                           \
        else gap[k] = ((double)best - (double)second) / (double)best;                  \
      }                                                                                \
      ipiv[k] = (int32_t)(piv + 1);                                                    \
      if (A[IDX(piv, k, lda)] == (T)0) {                                               \
        if (info == 0) info = (int)(k + 1);                                            \
        continue;                                                                      \
      }                                                                                \
      if (piv != k) {                                                                  \
        for (int64_t j = 0; j < n; ++j) {                                              \
          T t = A[IDX(k, j, lda)];                                                     \
          A[IDX(k, j, lda)] = A[IDX(piv, j, lda)];                                     \
          A[IDX(piv, j, lda)] = t;                                                     \
        }                                                                              \
      }                                                                                \
      T pivot = A[IDX(k, k, lda)];                                                     \
      for (int64_t i = k + 1; i < m; ++i) A[IDX(i, k, lda)] = A[IDX(i, k, lda)] / pivot; \
      UPDATE_LOOP(T)                                                                   \
    }                                                                                  \
    return info;                                                                       \
  }

/* rank-1 update of the trailing block; columns are independent, so the
 * threaded build splits them across threads without changing any value */
#ifdef _OPENMP
#define UPDATE_LOOP(T)                                                                 \
  _Pragma("omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if(nthreads > 1 && (m - k) * (n - k) > 65536)") \
  for (int64_t j = k + 1; j < n; ++j) {                                                \
    T u = A[IDX(k, j, lda)];                                                           \
    T* col = A + IDX(0, j, lda);                                                       \
    const T* l = A + IDX(0, k, lda);                                                   \
    for (int64_t i = k + 1; i < m; ++i) {                                              \
      T prod = l[i] * u;                                                               \
      col[i] = col[i] - prod;                                                          \
    }                                                                                  \
  }
#else
#define UPDATE_LOOP(T)                                                                 \
  for (int64_t j = k + 1; j < n; ++j) {                                                \
    T u = A[IDX(k, j, lda)];                                                           \
    T* col = A + IDX(0, j, lda);                                                       \
    const T* l = A + IDX(0, k, lda);                                                   \
    for (int64_t i = k + 1; i < m; ++i) {                                              \
      T prod = l[i] * u;                                                               \
      col[i] = col[i] - prod;                                                          \
    }                                                                                  \
  }
#endif

DEFINE_GETRF(double, oracle_dgetrf, fabs)
DEFINE_GETRF(float, oracle_sgetrf, fabsf)

/* Left-looking (column-at-a-time) variant: column j first receives all earlier
 * interchanges, then its updates from columns 0..j-1 in increasing order, then
 * its own pivot search, interchange and scaling.  Every element sees the same
 * ordered sequence of operations as in the right-looking loop. */
int oracle_dgetrf_left(int64_t m, int64_t n, double* A, int64_t lda, int32_t* ipiv) {
  int64_t p = m < n ? m : n;
  int info = 0;
  for (int64_t j = 0; j < n; ++j) {
    double* c = A + IDX(0, j, lda);
    int64_t kmax = j < p ? j : p;
    for (int64_t k = 0; k < kmax; ++k) {
      int64_t piv = ipiv[k] - 1;
      if (piv != k) { double t = c[k]; c[k] = c[piv]; c[piv] = t; }
    }
    for (int64_t k = 0; k < kmax; ++k) {
      if (A[IDX(k, k, lda)] == 0.0) continue; /* singular step: no update */
      double u = c[k];
      const double* l = A + IDX(0, k, lda);
      for (int64_t i = k + 1; i < m; ++i) {
        double prod = l[i] * u;
        c[i] = c[i] - prod;
      }
    }
    if (j < p) {
      int64_t piv = j;
      double best = fabs(c[j]);
      for (int64_t i = j + 1; i < m; ++i)
        if (fabs(c[i]) > best) { best = fabs(c[i]); piv = i; }
      ipiv[j] = (int32_t)(piv + 1);
      if (c[piv] == 0.0) {
        if (info == 0) info = (int)(j + 1);
        continue;
      }
      if (piv != j) /* interchange the rows in the already-factored columns and this one */
        for (int64_t jj = 0; jj <= j; ++jj) {
          double t = A[IDX(j, jj, lda)];
          A[IDX(j, jj, lda)] = A[IDX(piv, jj, lda)];
          A[IDX(piv, jj, lda)] = t;
        }
      double pivot = c[j];
      for (int64_t i = j + 1; i < m; ++i) c[i] = c[i] / pivot;
    }
  }
  return info;
}

/* Solve A X = B given the factors: apply the interchanges to B in order
 * k = 0..n-1, forward substitution with unit lower L, back substitution with
 * U; each sum runs in increasing index order.  Returns the first k+1 with
 * U(k,k) == 0 (and leaves B partly solved), else 0. */
#define DEFINE_GETRS(T, NAME)                                                          \
  int NAME(int64_t n, int64_t nrhs, const T* LU, int64_t lda, const int32_t* ipiv,    \
           T* B, int64_t ldb) {                                                        \
    for (int64_t k = 0; k < n; ++k)                                                    \
      if (LU[IDX(k, k, lda)] == (T)0) return (int)(k + 1);                             \
    for (int64_t r = 0; r < nrhs; ++r) {                                               \
      T* b = B + IDX(0, r, ldb);                                                       \
      for (int64_t k = 0; k < n; ++k) {                                                \
        int64_t piv = ipiv[k] - 1;                                                     \
        if (piv != k) { T t = b[k]; b[k] = b[piv]; b[piv] = t; }                       \
      }                                                                                \
      for (int64_t i = 0; i < n; ++i) {                                                \
        T s = b[i];                                                                    \
        for (int64_t k = 0; k < i; ++k) { T prod = LU[IDX(i, k, lda)] * b[k]; s = s - prod; } \
        b[i] = s;                                                                      \
      }                                                                                \
      for (int64_t i = n - 1; i >= 0; --i) {                                           \
        T s = b[i];                                                                    \
        for (int64_t k = i + 1; k < n; ++k) { T prod = LU[IDX(i, k, lda)] * b[k]; s = s - prod; } \
        b[i] = s / LU[IDX(i, i, lda)];                                                 \
      }                                                                                \
    }                                                                                  \
    return 0;                                                                          \
  }

DEFINE_GETRS(double, oracle_dgetrs)
DEFINE_GETRS(float, oracle_sgetrs)

/* Independent systems: factor and solve each (A_i packed column-major with
 * lda = n_i at A + a_off[i], b_i at B + b_off[i], pivots at ipiv + p_off[i]).
 * Systems are spread over threads; each system runs the sequential code. */
#define DEFINE_GESV_BATCHED(T, NAME, GETRF, GETRS)                                     \
  void NAME(int32_t batch, const int32_t* nvec, const int64_t* a_off, T* A,            \
            const int64_t* p_off, int32_t* ipiv, const int64_t* b_off, T* B,           \
            int32_t* info, int nthreads) {                                             \
    (void)nthreads;                                                                    \
    _Pragma("omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)") \
    for (int32_t s = 0; s < batch; ++s) {                                              \
      int64_t n = nvec[s];                                                             \
      int inf = GETRF(n, n, A + a_off[s], n, ipiv + p_off[s], NULL, -1, 1);           \
      info[s] = inf;                                                                   \
      if (inf == 0) GETRS(n, 1, A + a_off[s], n, ipiv + p_off[s], B + b_off[s], n);    \
    }                                                                                  \
  }

DEFINE_GESV_BATCHED(double, oracle_dgesv_batched, oracle_dgetrf, oracle_dgetrs)
DEFINE_GESV_BATCHED(float, oracle_sgesv_batched, oracle_sgetrf, oracle_sgetrs)

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
