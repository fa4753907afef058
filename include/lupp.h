/*
 * lupp -- LU factorization with partial pivoting on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every matrix, vector, pivot and info
 * pointer passed to a compute call is DEVICE memory owned by the caller; the
 * library never frees caller memory.  Matrices are column-major with a leading
 * dimension (lda >= max(1, rows)); all sizes and offsets are 64-bit.
 *
 * The problem statement follows the paper's notation: a dense real m x n
 * matrix A with submatrices A(c:d, e:f) (Section 2), factored in place
 * (Section 3.2 stores one matrix and overwrites it at every step), right-looking
 * one block of columns at a time with the column-block factorization as the
 * step every other step waits for (Section 4.1) and the loop written as
 * FLAME partition / repartition / continue-with (Section 4.3).  The paper does
 * not write LU out; the factorization computed is the textbook P*A = L*U with
 * partial pivoting and LAPACK's getrf/getrs conventions:
 *   - L is unit lower triangular and stored strictly below the diagonal of A;
 *     U is stored on and above it;
 *   - the pivot of column k is the FIRST row (lowest index) among those of
 *     maximal |a(i,k)|, i >= k;
 *   - ipiv[k] (1-based) is the row interchanged with row k at step k;
 *   - *info = 0, or the 1-based index of the first exactly zero pivot
 *     (the factorization still completes; that step does no elimination).
 *
 * Return codes: 0 = success; -i = argument i (1-based, the handle counts as
 * argument 1) is invalid and nothing was launched; > 0 = runtime failure
 * (LUPP_ERR_*).  Compute calls are asynchronous on the handle's stream;
 * numerical singularity is reported through *info, never through the return
 * code.  NaN or Inf inputs are outside the contract: calls terminate but the
 * results are unspecified.
 */
#ifndef LUPP_H
#define LUPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lupp_handle_st* lupp_handle_t;

enum {
  LUPP_OK = 0,
  LUPP_ERR_HIP = 1000,         /* 1000 + hipError_t of the failing runtime call   */
  LUPP_ERR_ALLOC = 2000,       /* workspace allocation failed                      */
  LUPP_ERR_INTERNAL = 2001,    /* a device-side bounded wait expired (reported by
                                  lupp_sync); results of the affected call invalid */
  LUPP_ERR_UNSUPPORTED = 2002  /* size or option outside what this build supports */
};

/* Options for lupp_set_option. */
enum {
  LUPP_OPT_NB = 1,         /* outer block size b of the right-looking loop (default 256)  */
  LUPP_OPT_PANEL_LEAF = 2, /* column width at which the recursive panel stops (8/16/32)    */
  LUPP_OPT_TIMING = 3,     /* 1: record HIP events around every phase of xGETRF (below)    */
  LUPP_OPT_LOOKAHEAD = 4   /* 1 (default): factor the next column block on a second stream
                              while the trailing update runs; 0: one stream, in order      */
};

/* Phases reported by lupp_timing_summary. */
enum {
  LUPP_PHASE_PANEL = 0,     /* recursive column-block factorization          */
  LUPP_PHASE_LASWP = 1,     /* interchanges applied outside the column block */
  LUPP_PHASE_TRSM = 2,      /* U12 := inv(L11) * A12                         */
  LUPP_PHASE_UPDATE = 3,     /* A22 := A22 - A21 * U12, every launch          */
  LUPP_PHASE_UPDATE_BIG = 4, /* the same, launches of the 128x128-tile kernel */
  LUPP_PHASE_PANEL_LEAF = 5, /* inside the column block: leaf factorizations  */
  LUPP_PHASE_PANEL_SWAP = 6, /* inside the column block: interchanges         */
  LUPP_PHASE_PANEL_TRSM = 7, /* inside the column block: triangular solves    */
  LUPP_PHASE_PANEL_GEMM = 8  /* inside the column block: updates              */
};

/* Create a handle on the current HIP device.  The handle owns its workspace
 * (allocated on first use, freed by lupp_destroy) and borrows a stream
 * (default: the null stream).  Errors: -1 if h is NULL. */
int lupp_create(lupp_handle_t* h);

/* Release the handle and its workspace.  Waits for the handle's stream. */
int lupp_destroy(lupp_handle_t h);

/* Borrow a hipStream_t (passed as void*) for subsequent calls; NULL = null stream. */
int lupp_set_stream(lupp_handle_t h, void* hip_stream);

/* Set an option (see LUPP_OPT_*).  Errors: -2 unknown option, -3 bad value. */
int lupp_set_option(lupp_handle_t h, int option, int64_t value);

/* Wait for all work on the handle's stream.  Returns LUPP_ERR_INTERNAL once if
 * a device-side wait of an earlier call expired, else 0 or LUPP_ERR_HIP+e. */
int lupp_sync(lupp_handle_t h);

/* Instrumentation (test and benchmark use).  With LUPP_OPT_TIMING set, every
 * xGETRF phase launched on the handle's stream is bracketed by HIP events on
 * that stream.  This call synchronizes the stream and returns, for one phase,
 * the number of recorded intervals, their summed duration (ms) and their
 * summed algorithmic flop count (2*M*N*K for the update, M*N*M for the
 * triangular solve, 0 otherwise); reset != 0 then clears all records.
 * Errors: -2 unknown phase, -3/-4/-5 NULL output. */
int lupp_timing_summary(lupp_handle_t h, int phase, int64_t* count, double* ms, double* flops, int reset);

/* Human-readable text for a return code (static storage). */
const char* lupp_status_string(int status);

/*
 * xGETRF: P*A = L*U of an m x n matrix, in place.
 *   m, n   >= 0
 *   dA     device, column-major, lda >= max(1, m); overwritten by L\U
 *   dipiv  device int32[min(m,n)]: 1-based interchanges, k+1 <= ipiv[k] <= m
 *   dinfo  device int32[1]: 0, or the first k (1-based) with U(k,k) == 0
 * Blocked right-looking: per block of b columns, the column block is factored
 * (pivot search, interchanges, scaling, rank updates; recursive), the block's
 * interchanges are applied to the other columns, U12 := inv(L11)*A12 and
 * A22 := A22 - A21*U12 (the paper's finding that the matrix-matrix products
 * dominate: Sections 4.1 and 5.4).
 * Requires m < 2^31 (ipiv is int32).  Errors: -2 m, -3 n, -4 dA, -5 lda,
 * -6 dipiv, -7 dinfo.
 */
int lupp_dgetrf(lupp_handle_t h, int64_t m, int64_t n, double* dA, int64_t lda,
                int32_t* dipiv, int32_t* dinfo);
int lupp_sgetrf(lupp_handle_t h, int64_t m, int64_t n, float* dA, int64_t lda,
                int32_t* dipiv, int32_t* dinfo);

/*
 * xGETRS: solve A*X = B with the factors from xGETRF (square n x n).
 *   trans  'N' only (transposed solves are not provided; -2 otherwise)
 *   dLU    device, lda >= max(1,n);  dipiv device int32[n]
 *   dB     device n x nrhs, ldb >= max(1,n); overwritten by X
 * X = inv(U) * inv(L) * P * B: the interchanges are applied in order, then the
 * unit-lower and upper triangular solves.  No singularity check (a zero U(k,k)
 * yields Inf/NaN, as in LAPACK's getrs); check *info from xGETRF first.
 * Errors: -2 trans, -3 n, -4 nrhs, -5 dLU, -6 lda, -7 dipiv, -8 dB, -9 ldb.
 */
int lupp_dgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const double* dLU,
                int64_t lda, const int32_t* dipiv, double* dB, int64_t ldb);
int lupp_sgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const float* dLU,
                int64_t lda, const int32_t* dipiv, float* dB, int64_t ldb);

#ifdef __cplusplus
}
#endif

#endif /* LUPP_H */
