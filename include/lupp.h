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
  LUPP_ERR_INTERNAL = 2001,    /* a device-side bounded wait expired, or the
                                  triangular solve's block tickets were out of step
                                  (reported by lupp_sync); results of the affected
                                  call invalid */
  LUPP_ERR_UNSUPPORTED = 2002, /* size or option outside what this build supports */
  LUPP_ERR_SINGULAR = 2003     /* xGETRS was given a U with an exactly zero diagonal
                                  entry (reported by lupp_sync)                    */
};

/* Options for lupp_set_option. */
enum {
  LUPP_OPT_NB = 1,         /* outer block size b of the right-looking loop (default 512)  */
  LUPP_OPT_PANEL_LEAF = 2, /* widest column block factored in one cooperative launch
                              (16 .. 256, a multiple of 16; default 64); wider blocks
                              split recursively with a triangular solve and a GEMM      */
  LUPP_OPT_TIMING = 3,     /* 1: record HIP events around every phase of xGETRF (below);
                              2: around the trailing updates only (LUPP_PHASE_UPDATE and
                              LUPP_PHASE_UPDATE_BIG), which leaves the latency-bound
                              column-block chain uninstrumented                           */
  LUPP_OPT_LOOKAHEAD = 4,  /* lookahead depth d (0..16).  1 (default): factor the next
                              column block on a second stream while the trailing update
                              runs; 0: one stream, in order.  d >= 2: the dataflow
                              (algorithm-by-blocks) runtime: the loop becomes tasks on
                              column blocks whose dependencies are derived from the blocks
                              each task reads and writes, issued onto CU-partitioned
                              streams with event waits, the column-block chain free to run
                              up to d steps ahead of the large updates (the paper's
                              Sections 4.1 and 4.4).  Factors and pivots are identical for
                              every d.  d >= 2 needs the deferred interchanges (below);
                              where they do not apply, d = 1 is used                       */
  LUPP_OPT_UPDATE_PREC = 5, /* lupp_sgetrf only: format of the operands of the trailing
                              update A22 -= A21*U12, one of LUPP_PREC_* (default FP32).  The
                              column-block factorization and U12 stay FP32; the products are
                              accumulated in FP32 and A22 is stored in FP32.               */
  LUPP_OPT_DEFER_SWAPS = 6, /* 1 (default): the interchanges of every step reach the finished
                              columns on its left once, at the end, composed into one row
                              permutation per column block (same result, one pass instead
                              of one per step; needs a workspace of about 2*m*n/nb bytes,
                              nb <= 512 and m - nb <= 32768 for FP64 or 65536 for FP32,
                              otherwise ignored); 0: at every step, as in LAPACK            */
  LUPP_OPT_SPLIT_UPDATE = 7, /* 1 (default, with lookahead): once the next column block is
                              factored, its CUs take the last columns of the remaining
                              update (sized from the measured panel time and GEMM rate, so
                              that both shares end together); 0: the bulk CUs take it all.
                              FP64/FP32 results are identical either way                 */
  LUPP_OPT_LP_PACKED = 8    /* with a low-precision update format: 1 (default): each update
                              scales and rounds A21 and U12 once into a handle workspace in
                              the matrix cores' operand order (4 slots of about
                              2*(m+n)*nb bytes, for updates that run concurrently), and the
                              GEMM streams them; 0: every tile of the GEMM rounds its FP32
                              operands while staging them.  Identical results either way  */
};

/* Operand formats of the trailing update (LUPP_OPT_UPDATE_PREC) and of the
 * factorization inside lupp_dgesv_mixed.  FP16 and FP8 multiply every 128-row
 * block of A21 and every 128-column block of U12 by a power of two so that its
 * largest magnitude lands just under the format's largest finite value (65504,
 * 448) before rounding; the scales are exact and are undone in FP32. */
enum {
  LUPP_PREC_FP32 = 0,
  LUPP_PREC_BF16 = 1,  /* bfloat16, round to nearest even, unscaled             */
  LUPP_PREC_FP16 = 2,  /* IEEE binary16, round to nearest even, block-scaled     */
  LUPP_PREC_FP8_E4M3 = 3 /* OCP FP8 e4m3, round to nearest even with saturation, block-scaled */
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
 * (default: the null stream).  Creation itself allocates no device memory: it
 * looks up the device address of lupp_dgesv_batched_noalloc's scratch array
 * on this device.  The first batched call on a handle creates the handle's
 * class streams and events (no device memory).
 * Errors: -1 if h is NULL. */
int lupp_create(lupp_handle_t* h);

/* Release the handle and its workspace.  Waits for the handle's stream. */
int lupp_destroy(lupp_handle_t h);

/* Borrow a hipStream_t (passed as void*) for subsequent calls; NULL = null stream. */
int lupp_set_stream(lupp_handle_t h, void* hip_stream);

/* Set an option (see LUPP_OPT_*).  Errors: -2 unknown option, -3 bad value. */
int lupp_set_option(lupp_handle_t h, int option, int64_t value);

/* Wait for all work on the handle's streams and collect the device-side status
 * of the calls made since the previous lupp_sync.  Returns, in this order of
 * precedence: LUPP_ERR_HIP+e if the wait itself failed; LUPP_ERR_INTERNAL if a
 * bounded wait of the column-block kernel or of the triangular solve expired,
 * or the solve found its block tickets out of step (the affected results are
 * invalid; the flags are cleared and the solve's ticket count re-read from the
 * device, so later calls run normally); LUPP_ERR_SINGULAR if an xGETRS met an
 * exactly zero U(k,k) (its X holds Inf/NaN); else 0.  Each status is reported
 * once. */
int lupp_sync(lupp_handle_t h);

/* Device workspace, in bytes, that the handle holds after a call of kind op
 * with the handle's current options (allocated on the call's first use, kept
 * and reused until lupp_destroy; an upper bound for the mixed solve).
 *   LUPP_WS_DGETRF / LUPP_WS_SGETRF: an m x n factorization;
 *   LUPP_WS_DGETRS / LUPP_WS_SGETRS: a solve of order n (m ignored);
 *   LUPP_WS_DGESV_MIXED: a mixed solve of order n with GMRES restart length k
 *     (k = 1 for classical refinement; m ignored);
 *   LUPP_WS_BATCHED: a batched call of m systems (n ignored).
 * Host only; nothing is allocated.  Errors: -2 op, -3 m, -4 n, -5 k,
 * -6 bytes NULL. */
enum {
  LUPP_WS_DGETRF = 1,
  LUPP_WS_SGETRF = 2,
  LUPP_WS_DGETRS = 3,
  LUPP_WS_SGETRS = 4,
  LUPP_WS_DGESV_MIXED = 5,
  LUPP_WS_BATCHED = 6
};
int lupp_workspace_bytes(lupp_handle_t h, int op, int64_t m, int64_t n, int64_t k, size_t* bytes);

/* Test hook for the error paths of lupp_sync; not for production use.  Makes
 * no kernel wait or fault: what = 1 sets the triangular solve's device error
 * flag as an expired wait would; what = 2 moves the host's ticket count of the
 * triangular solve far ahead of the device counter, so that every workgroup of
 * the next solve finds its ticket out of range, writes nothing and exits at
 * once (x is left as the interchanges made it).  Either is reported by the
 * next lupp_sync as LUPP_ERR_INTERNAL.  Errors: -2 what. */
int lupp_test_inject_fault(lupp_handle_t h, int what);

/* Instrumentation (test and benchmark use).  With LUPP_OPT_TIMING set, every
 * xGETRF phase launched on the handle's stream is bracketed by HIP events on
 * that stream.  This call synchronizes the stream and returns, for one phase,
 * the number of recorded intervals, their summed duration (ms) and their
 * summed algorithmic flop count (2*M*N*K for the update, M*N*M for the
 * triangular solve, 0 otherwise); reset != 0 then clears all records.
 * Errors: -2 unknown phase, -3/-4/-5 NULL output. */
int lupp_timing_summary(lupp_handle_t h, int phase, int64_t* count, double* ms, double* flops, int reset);

/* Instrumentation: the summed algorithmic bytes of the intervals recorded for
 * a phase since the last reset (the updates: C read and written once, A and B
 * read once; 0 for phases without such a count).  Host only; call before the
 * lupp_timing_summary that resets.  Errors: -2 unknown phase, -3 NULL. */
int lupp_timing_bytes(lupp_handle_t h, int phase, double* bytes);

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
 * Size limit: m <= 131072 (the column-block kernel runs one workgroup of
 * 1024 threads per 1024 rows, at most 128 workgroups); larger m returns
 * LUPP_ERR_UNSUPPORTED before anything is launched.
 * Co-residency: the column-block kernel's workgroups exchange pivot records
 * through device memory and wait for each other, so they must all be resident
 * at once.  It is launched with at most one workgroup per CU of the stream it
 * runs on: with lookahead, on a stream masked to 32 CUs (m - k <= 32768 rows
 * left) or 64 CUs (<= 65536), otherwise on the caller's stream (up to 128
 * workgroups on the device's 256 CUs).  Work the caller runs concurrently on
 * the same GPU may delay but not prevent residency; every wait is bounded, and
 * an expired wait is reported as LUPP_ERR_INTERNAL by lupp_sync instead of
 * hanging.
 * Errors: -2 m (negative or >= 2^31), -3 n, -4 dA, -5 lda, -6 dipiv, -7 dinfo.
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
 * unit-lower and upper triangular solves.  The diagonal of U is checked on the
 * device: an exactly zero U(k,k) still completes the call (X then holds
 * Inf/NaN, as in LAPACK's getrs) and is reported as LUPP_ERR_SINGULAR by the
 * next lupp_sync.  Asynchronous on the handle's stream.
 * Errors: -2 trans, -3 n, -4 nrhs, -5 dLU, -6 lda, -7 dipiv, -8 dB, -9 ldb.
 */
int lupp_dgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const double* dLU,
                int64_t lda, const int32_t* dipiv, double* dB, int64_t ldb);
int lupp_sgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const float* dLU,
                int64_t lda, const int32_t* dipiv, float* dB, int64_t ldb);

/*
 * Mixed-precision solve with FP64 iterative refinement.
 *
 * The paper factors in FP64 only; this entry point extends the same blocked
 * factorization (the column-block step and the dominant matrix-matrix update
 * of Sections 4.1 and 5.4) with cheaper update formats, and recovers FP64
 * accuracy with iterative refinement in the textbook form (Higham, Accuracy
 * and Stability of Numerical Algorithms, 2nd ed., Ch. 12) and its
 * GMRES-preconditioned variant (Carson and Higham, SIAM J. Sci. Comput. 40,
 * 2018).
 *
 * The FP64 matrix A (n x n, not modified) is rounded to FP32 and factored with
 * lupp_sgetrf, the trailing updates taking their operands in opts->factor_prec
 * (FP32 accumulation and storage).  Each right-hand side is then refined in
 * FP64 against the original A:
 *   r = b - A x (FP64), eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf),
 * stopping when eta <= opts->tol.  The correction d solves A d = r:
 *   LUPP_IR_CLASSICAL: d = inv(U) inv(L) P r with the FP32 factors;
 *   LUPP_IR_GMRES: d from restarted GMRES in FP64 on the left-preconditioned
 *     system inv(U) inv(L) P A d = inv(U) inv(L) P r (one cycle of at most
 *     gmres_restart Arnoldi steps per outer iteration, classical Gram-Schmidt
 *     applied twice, stopped at relative preconditioned residual inner_tol).
 * x starts at 0, so the first correction is the plain low-precision solve.
 * Stopping: CONVERGED when eta <= tol; DIVERGED when eta is NaN or grows above
 * 10x the best value so far; STAGNATED when eta fails to halve over two
 * iterations; MAXITER after max_iter outer iterations.  On any stop other than
 * CONVERGED, dX holds the iterate with the smallest eta.  With fallback_fp64
 * set, a non-converged system is solved again with lupp_dgetrf/lupp_dgetrs on
 * an FP64 copy and the report says so.
 *
 *   dA  device FP64 n x n, lda >= max(1,n), read only
 *   dB  device FP64 n x nrhs, ldb >= max(1,n), read only
 *   dX  device FP64 n x nrhs, ldx >= max(1,n), written
 *   opts  host, NULL = defaults (lupp_ir_opts_default); rep host, may be NULL
 * The call allocates its workspace (FP32 copy of A and O(n * gmres_restart)
 * vectors) in the handle, keeps it for later calls, and returns after the
 * work is done (it synchronizes the handle's stream).  The report aggregates
 * over the right-hand sides: the worst status, the largest eta, the largest
 * outer and the summed inner iteration counts.
 * Errors: -2 n, -3 nrhs, -4 dA, -5 lda, -6 dB, -7 ldb, -8 dX, -9 ldx,
 * -10 opts out of range.
 */
enum { LUPP_IR_CLASSICAL = 0, LUPP_IR_GMRES = 1 };
enum {
  LUPP_IR_CONVERGED = 0,
  LUPP_IR_STAGNATED = 1,
  LUPP_IR_DIVERGED = 2,
  LUPP_IR_SINGULAR = 3, /* the FP32 factorization met an exactly zero pivot */
  LUPP_IR_MAXITER = 4
};

typedef struct lupp_ir_opts {
  int32_t factor_prec;        /* LUPP_PREC_*                              (FP16)  */
  int32_t solver;             /* LUPP_IR_CLASSICAL or LUPP_IR_GMRES   (GMRES)     */
  double tol;                 /* target backward error                  (1e-14)  */
  int32_t max_iter;           /* outer iterations, 1..1000 (50 classical, 10 GMRES) */
  int32_t gmres_restart;      /* Arnoldi steps per GMRES cycle, 1..60      (30)   */
  double inner_tol;           /* GMRES relative residual target          (1e-6)  */
  int64_t nb;                 /* block size of the factorization, 0 = handle's   */
  int32_t fallback_fp64;      /* 1: re-solve non-converged systems in FP64  (0)  */
} lupp_ir_opts;

typedef struct lupp_ir_report {
  int32_t status;             /* LUPP_IR_*                                        */
  int32_t iters;              /* outer iterations (largest over the RHS)          */
  int32_t inner_iters;        /* GMRES steps (sum over the RHS)                   */
  int32_t info;               /* info of the FP32 factorization                    */
  int32_t fallback_used;      /* number of RHS solved again in FP64               */
  double backward_error;      /* final eta (largest over the RHS)                 */
  double factor_ms;           /* FP64->FP32 rounding and factorization             */
  double refine_ms;           /* refinement of all right-hand sides                */
} lupp_ir_report;

/* Fill *opts with the defaults above for the given solver. */
void lupp_ir_opts_default(lupp_ir_opts* opts, int32_t solver);

int lupp_dgesv_mixed(lupp_handle_t h, int64_t n, int64_t nrhs, const double* dA, int64_t lda,
                     const double* dB, int64_t ldb, double* dX, int64_t ldx,
                     const lupp_ir_opts* opts, lupp_ir_report* rep);

/*
 * Batched factorization and solve of many independent small systems.
 *
 * The paper's factorizations are of one large matrix; this entry point
 * applies the same factorization (partial pivoting, LAPACK conventions, the
 * elimination step of Section 4.1 taken one column at a time) to a batch of
 * small systems at once, one workgroup per system with the system held in
 * registers, scheduled by size class as the handle's schedule says
 * (lupp_batched_set_schedule below).
 *
 *   batch       number of systems (>= 0)
 *   dn          device int32[batch]: order n_i of system i, 0 <= n_i <= 128
 *   dA, dA_off  device: system i is the column-major n_i x n_i matrix at
 *               dA + dA_off[i] (leading dimension n_i), overwritten by L\U
 *   dipiv, dipiv_off  device: ipiv of system i at dipiv + dipiv_off[i]
 *               (n_i int32 entries, 1-based, LAPACK convention)
 *   dB, dB_off  device: right-hand side of system i (n_i entries) at
 *               dB + dB_off[i], overwritten by the solution x_i
 *   dinfo       device int32[batch]: 0; k > 0 when U(k,k) of system i is
 *               exactly zero (the factorization completes, x_i is not
 *               computed and b_i is left unchanged, as in LAPACK's gesv);
 *               -1 when n_i is outside [0, 128] (system untouched);
 *               -1000 if the workgroup's internal step schedule stalled
 *               (bounded waits; a fault in the library, never expected):
 *               system i's outputs are then not written
 * Systems must not overlap.  The call is asynchronous on the handle's
 * stream; it allocates its workspace on the first call for a batch size and
 * afterwards neither allocates nor synchronizes with the host, so it can be
 * captured in a HIP graph.  Host-side errors: -2 batch, then the pointer
 * arguments in order (-3 dn ... -10 dinfo; for xGETRF_BATCHED -8 dinfo).
 */
int lupp_dgesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                       double* dA, const int64_t* dipiv_off, int32_t* dipiv,
                       const int64_t* dB_off, double* dB, int32_t* dinfo);
int lupp_sgesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                       float* dA, const int64_t* dipiv_off, int32_t* dipiv,
                       const int64_t* dB_off, float* dB, int32_t* dinfo);
/*
 * Allocation-free variant of lupp_dgesv_batched, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * lupp_dgesv_batched, but the class list and counters live in a fixed array
 * of the library (about 4 MiB per device, held until the process ends)
 * instead of handle workspace, so no call allocates or frees device memory
 * (the handle's first batched call creates its class streams, which is not a
 * device allocation; a caller that captures graphs can make a first call
 * outside the capture).
 *   batch <= 1048576 (LUPP_NOALLOC_MAX_BATCH); a larger batch returns
 *   LUPP_ERR_UNSUPPORTED before anything is launched.
 * Every call on one device shares that device's array: calls that may
 * overlap in time on the same device (different handles or streams without
 * ordering between them) race and corrupt each other's results.  Calls
 * ordered on one stream do not.  Nothing in the array needs clearing: each
 * call rewrites the parts it reads.
 * Errors: as lupp_dgesv_batched.
 */
#define LUPP_NOALLOC_MAX_BATCH 1048576
int lupp_dgesv_batched_noalloc(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                               double* dA, const int64_t* dipiv_off, int32_t* dipiv,
                               const int64_t* dB_off, double* dB, int32_t* dinfo);

/*
 * Schedules of the batched calls, and the autotuner that chooses them.
 *
 * The systems of a batched call are sorted into size classes by their order
 * (class c holds the orders in (nmax[c-1], nmax[c]], nmax[-1] = 0); each class
 * is one persistent launch of a kernel shape (wavefronts per system, rows per
 * lane slot group, columns per wavefront) with a grid of grid_pct percent of
 * the workgroups of that shape that fit on the device at once.  The classes
 * run concurrently on streams of the handle.  Every shape computes the same
 * factors, pivots and solutions bit for bit; schedules differ only in speed.
 * Each handle holds one schedule for FP64 (fp32 = 0) and one for FP32
 * (fp32 = 1), initially four classes (orders <= 32, 64, 96, 128).  The
 * package's autotuner (paper_2104_05782_amd/autotune.py) chooses schedules by
 * timing HIP-graph replays of the batched call over candidate class splits,
 * shapes and grids, and keeps its choice per GPU architecture.
 */
#define LUPP_BATCH_MAX_CLASSES 6
typedef struct lupp_batched_schedule {
  int32_t nclass;                             /* 1 .. LUPP_BATCH_MAX_CLASSES       */
  int32_t nmax[LUPP_BATCH_MAX_CLASSES];       /* increasing; nmax[nclass-1] = 128 */
  int32_t shape[LUPP_BATCH_MAX_CLASSES];      /* 0 .. lupp_batched_shape_count()-1,
                                                 holding orders up to nmax[c]    */
  int32_t grid_pct[LUPP_BATCH_MAX_CLASSES];   /* 1 .. 100                         */
} lupp_batched_schedule;

/* Number of compiled kernel shapes, and shape v's geometry: wavefronts per
 * system, row capacity (64 or 128), columns per wavefront, largest order it
 * holds.  Host only.  lupp_batched_shape returns -1 for v out of range. */
int lupp_batched_shape_count(void);
int lupp_batched_shape(int32_t v, int32_t* nw, int32_t* rows, int32_t* cols, int32_t* nmax);

/* The handle's schedule for FP64 (fp32 = 0) or FP32 (fp32 = 1).  set with
 * s = NULL restores the initial schedule.  A schedule takes effect for calls
 * made after it is set.  Errors: -2 fp32, -3 out NULL (get) or an invalid
 * schedule (set: bounds not increasing or not ending at 128, a shape that
 * cannot hold its class, grid_pct outside 1..100). */
int lupp_batched_get_schedule(lupp_handle_t h, int32_t fp32, lupp_batched_schedule* out);
int lupp_batched_set_schedule(lupp_handle_t h, int32_t fp32, const lupp_batched_schedule* s);

/* Factorization only (no right-hand sides). */
int lupp_dgetrf_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                        double* dA, const int64_t* dipiv_off, int32_t* dipiv, int32_t* dinfo);
int lupp_sgetrf_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                        float* dA, const int64_t* dipiv_off, int32_t* dipiv, int32_t* dinfo);

/*
 * Householder QR factorization A = Q R of an m x n FP64 matrix, in place
 * (the paper's HQR, Section 2.2: R upper triangular, V unit lower triangular
 * holding the Householder vectors, one scalar per vector), blocked with the
 * compact WY form of Section 2.3.  Conventions of LAPACK's dgeqrf:
 *   - reflector j is H_j = I - tau_j v_j v_j^T with v_j[j] = 1, v_j zero above
 *     row j; it maps column j's entries from row j down to beta e_j with
 *     beta = -sign(alpha) ||x||_2 (sign(0) = +1); tau_j = 0 (H_j = I) when the
 *     entries below the diagonal are already zero;
 *   - on return R is on and above the diagonal of A, v_j[j+1:] below it, and
 *     Q = H_1 H_2 ... H_k, k = min(m, n);
 *   - dtau: device double[k].
 * Per block of 32 columns: the block's reflectors (one cooperative launch,
 * one exchange between workgroups per column), T with H_1 ... H_b =
 * I - V T V^T, and the trailing columns A2 := A2 - V (T^T (V^T A2)) as matrix
 * products; the columns right of each 128-column outer block get one such
 * update with its 128 reflectors.  With LUPP_OPT_LOOKAHEAD >= 1 (default),
 * large steps factor the next outer block on the handle's CU-partitioned
 * streams while the rest of the update runs beside it (same result, bit for
 * bit); that work is joined back into the handle's stream before the call's
 * last operation, so ordering on the handle's stream and lupp_sync cover it.
 * Sums of squares are formed without scaling: entries whose squares
 * overflow are outside the contract.  Asynchronous on the handle's stream;
 * the column-block kernel's workgroups wait for each other (bounded waits, an
 * expiry reported by lupp_sync as LUPP_ERR_INTERNAL).
 * Size limit: m <= 131072 (LUPP_ERR_UNSUPPORTED beyond).
 * Errors: -2 m, -3 n, -4 dA, -5 lda, -6 dtau.
 */
int lupp_dgeqrf(lupp_handle_t h, int64_t m, int64_t n, double* dA, int64_t lda, double* dtau);

/*
 * Randomized UTV factorization (randUTV, the paper's Section 3.2) of a square
 * n x n FP64 matrix: A = U T V^T with U, V orthogonal and T upper triangular,
 * built b = 64 columns at a time.  With T22 = T[k0:, k0:] at step i
 * (k0 = 64 i):
 *   1. Y = (T22^T T22)^q T22^T G_i, G_i = G[k0:, k0:k0+64] (the Gaussian draws
 *      are an input: G is n x n, device); Householder QR of Y (as
 *      lupp_dgeqrf); T[:, k0:] and V[:, k0:] multiplied by its Q from the
 *      right;
 *   2. Householder QR of T22's first 64 columns, Q^T applied to T22 (entries
 *      below the diagonal become exactly 0), U[:, k0:] times Q;
 *   3. SVD of the 64 x 64 diagonal block (one-sided Jacobi, singular values in
 *      decreasing order): the block becomes diag(sigma), Us^T multiplies the
 *      block row right of it, Vs the block column above it, U and V get Us
 *      and Vs.
 * The last step, with at most 64 columns left, is step 3 on the whole block.
 * The diagonal of T approximates the singular values of A (the better, the
 * larger q).
 *   dA  device n x n, lda >= max(1, n): A on entry, T on return
 *   q   power steps, 0 .. 16
 *   dG  device n x n, ldg >= max(1, n), read only
 *   dU, dV  device n x n (ldu, ldv >= max(1, n)), written; either may be NULL
 *           (that factor is then not formed)
 * Singular vectors of each small SVD are fixed up to sign, so T's rows and
 * columns and U's and V's columns are determined up to sign.  Asynchronous on
 * the handle's stream.  Each step's SVD and the products with it run on a
 * second stream of the handle, and the products of U and V with the
 * Householder factors on a third; both are joined back into the handle's
 * stream before the call's last operation, so ordering on the handle's stream
 * and lupp_sync cover them.  Workspace in the handle: about 14 n x 64 + 3 n x 128
 * values beside the QR path's.  Size limit: n <= 131072.
 * Errors: -2 n, -3 dA, -4 lda, -5 q, -6 dG, -7 ldg, -9 ldu, -11 ldv.
 */
int lupp_drandutv(lupp_handle_t h, int64_t n, double* dA, int64_t lda, int32_t q, const double* dG, int64_t ldg,
                  double* dU, int64_t ldu, double* dV, int64_t ldv);

#ifdef __cplusplus
}
#endif

#endif /* LUPP_H */
