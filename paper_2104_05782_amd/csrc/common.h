// Internal declarations shared by the lupp HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lupp.h"

namespace lupp {

// ---------------------------------------------------------------- MFMA traits
// v_mfma_*_16x16x4: operand "a" lane l holds X[l%16][l/16] (16x4), operand "b"
// lane l holds Y[l/16][l%16] (4x16).  The GEMM feeds a = B-fragment and
// b = A-fragment, so the 16x16 result is C^T: lane l then holds C rows l%16
// (16 consecutive rows: coalesced column segments) and the column given by
// col(l, r) -- the FP64 and FP32 instructions place their four result
// registers differently (measured on gfx950).
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------- workspace
// Device-resident state of the cooperative panel kernel.  Per column and
// workgroup a record of 64-bit words, each carrying the column's tag in its
// upper half and 32 payload bits in its lower half: the candidate |a| (two
// words), its row (one word) and the candidate row (two words per value); a
// reader accepts a record word only when its tag is the current one, so no
// separate flag or store fence is needed.  Records are double-buffered by
// column parity.  The error flag is set when a bounded wait expires.
constexpr int kLeafMaxGroups = 128;
constexpr int kLeafMaxWidth = 16;
constexpr int kLeafRecWords = 3 + 2 * kLeafMaxWidth;  // 35 used
constexpr int kLeafRecStride = 36;

struct LeafSlots {
  uint32_t flags[kLeafMaxGroups];  // per-workgroup barrier tags of the column-block kernel
  int32_t err;                     // set when a bounded wait expires
  uint32_t uflag;                  // tag: workgroup 0 has published a chunk's U12 rows
  int32_t pad_[30];
  uint64_t rec[2][kLeafMaxGroups][kLeafRecStride];  // candidate records, by column parity
  uint64_t rowj[2][2 * kLeafMaxWidth];              // the diagonal row before the interchange
};

// Exchange records of the Householder panel kernel: per column (by parity)
// and workgroup 64 tagged words carrying 32 partial sums as 32-bit halves,
// and the diagonal row (32 values) published by workgroup 0.
constexpr int kQrMaxGroups = 256;
struct QrSlots {
  int32_t err;  // set when a bounded wait expires
  int32_t pad_[63];
  uint64_t rec[2][kQrMaxGroups][64];
  uint64_t rowj[2][64];
};

// Row movement of a run of consecutive interchanges k1..k2-1 (k2 - k1 <=
// kMaxSwaps), composed into one permutation: after the run, row dst[q] holds
// what row src[q] held before it.  The first k2 - k1 entries are the rows
// k1..k2-1 in order; the rest are the rows below k2 that the run touched.
constexpr int kMaxSwaps = 512;
struct SwapPairs {
  int32_t count;
  int32_t pad_[63];
  int32_t dst[2 * kMaxSwaps];
  int32_t src[2 * kMaxSwaps];
};

// ---------------------------------------------------------------- launchers
// C[M x N] -= A[M x K] * B[K x N], column-major (A, B and C must not overlap).
// *tile_out (optional) receives the tile configuration used: 0 = 128x32,
// 1 = 128x128, 2 = 64x64, -1 = nothing launched.  role: 0 a trailing update,
// 1 the share of an update run on the panel's CUs (128x128 tiles down to 32
// tiles), 2 a product inside the column-block or triangular-solve recursion;
// the FP64 kernel is named by it.
template <typename T>
hipError_t gemm_sub(hipStream_t s, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda,
                    const T* B, int64_t ldb, T* C, int64_t ldc, int* tile_out = nullptr, int role = 2);

// Factor the r x w column block P (leading dimension ld, w <= kBlockMaxWidth,
// r >= w) whose first row and column are the global row/column k: partial
// pivoting column by column in one cooperative launch, the interchanges
// applied across the w columns of the block and also to the columns P[:, c]
// for c in [oc_lo, 0) and [w, oc_hi) (the rest of the enclosing column
// block).  Writes ipiv[k + j] = k + piv + 1 and, on the first exactly zero
// pivot, *info.  Uses block_tags(w) consecutive tags from epoch.
constexpr int kBlockMaxWidth = 256;
template <typename T>
hipError_t panel_block(hipStream_t s, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k,
                       int32_t* info, LeafSlots* ws, uint32_t epoch, int64_t oc_lo, int64_t oc_hi);
uint32_t block_tags(int w);

// Number of cooperating workgroups panel_block uses for r rows.
int panel_groups(int64_t r);

// Triangular solve, one thread per right-hand column kept in registers
// (w <= 64): lower = unit lower (forward), else non-unit upper (backward).
template <typename T>
hipError_t trsm_small(hipStream_t s, bool lower, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B,
                      int64_t ldb);

// Compose interchanges k1..k2-1 (ipiv, 1-based rows of an m-row matrix) into
// *pairs (one workgroup).
hipError_t swap_pairs(hipStream_t s, const int32_t* ipiv, int64_t k1, int64_t k2, int64_t m, SwapPairs* pairs);

// Apply *pairs to columns [c0, c1) of A except the columns [skip0, skip1).
template <typename T>
hipError_t apply_pairs(hipStream_t s, T* A, int64_t lda, int64_t c0, int64_t c1, int64_t skip0, int64_t skip1,
                       const SwapPairs* pairs, int64_t max_pairs);

// Apply interchanges k1..k2-1 (ipiv, 1-based rows of the m-row matrix A) to
// columns [c0, c1) of A except the columns [skip0, skip1): swap_pairs then
// apply_pairs (k2 - k1 <= kMaxSwaps), or one thread per column for longer runs.
template <typename T>
hipError_t laswp(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t c0, int64_t c1, int64_t skip0, int64_t skip1,
                 const int32_t* ipiv, int64_t k1, int64_t k2, SwapPairs* pairs);

// Deferred interchanges of the finished columns.  Block j (columns
// [j*nb, (j+1)*nb), j < J-1) is left alone by the later steps j+1..J-1 of the
// loop; its rows [(j+1)*nb, m) are permuted once, at the end, by the
// composition of those steps' pairs: row i receives the row gmap_j(i), where
// gmap_j = h_{j+1} o ... o h_{J-1} and h_s maps dst -> src of step s's pairs.
// The maps of all blocks are stored back to back: block j's starts at
// j*m - nb*j*(j+1)/2 and has m - (j+1)*nb entries.
constexpr int kLeftGatherThreads = 1024;
// rows of a column held in registers by one workgroup: 32 (FP64) or 64 (FP32) per thread
__host__ __device__ inline int64_t left_gather_max_rows(size_t elem) {
  return (elem == 8 ? 32 : 64) * (int64_t)kLeftGatherThreads;
}
__host__ __device__ inline int64_t left_map_offset(int64_t j, int64_t m, int64_t nb) { return j * m - nb * j * (j + 1) / 2; }
__host__ __device__ inline int64_t left_map_entries(int64_t J, int64_t m, int64_t nb) { return J < 2 ? 0 : left_map_offset(J - 1, m, nb); }
// pairs[s], s < J: the composed pairs of step s.  g: 2*m ints of scratch.
hipError_t left_maps(hipStream_t s, const SwapPairs* pairs, int64_t J, int64_t m, int64_t nb, int32_t* g,
                     int32_t* gmap);
// Columns [0, (J-1)*nb) of A: rows [(j+1)*nb, m) of block j gathered by gmap_j
// (m - nb <= left_gather_max_rows(sizeof(T))).
template <typename T>
hipError_t left_gather(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t nb, int64_t J, const int32_t* gmap);

// B (w x ncols) := inv(L) * B, L unit lower triangular of order w <= kTrsmBandMaxW,
// in one launch (16 columns per workgroup).
constexpr int kTrsmBandMaxW = 256;
template <typename T>
hipError_t trsm_lower_band(hipStream_t s, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B, int64_t ldb);

// Triangular solve on a w x ncols block (w <= 64): lower=true solves with a
// unit lower triangle (forward), lower=false with a non-unit upper triangle.
template <typename T>
hipError_t trsm_leaf(hipStream_t s, bool lower, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B,
                     int64_t ldb);

// ---------------------------------------------------------------- mixed precision
// Number of int slots gemm_lp_sub needs as scale workspace for an M x N update.
int64_t gemm_lp_scale_slots(int64_t M, int64_t N);

// Bytes of the packed-operand workspace of an M x N x K low-precision update.
size_t gemm_lp_pack_bytes(int64_t M, int64_t N, int64_t K);

// C (FP32) -= A * B with A and B rounded to a low format: mode 1 = BF16,
// 2 = FP16, 3 = FP8 e4m3 (2 and 3 scale each 128-row block of A and 128-column
// block of B by a power of two first, using scale_ws).  With a packing
// workspace of at least gemm_lp_pack_bytes(M, N, K) bytes the operands are
// rounded once into it; otherwise each tile rounds them while staging.  Both
// give the same result bits.
hipError_t gemm_lp_sub(hipStream_t s, int mode, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float* C, int64_t ldc, int* scale_ws, void* pack,
                       size_t pack_bytes);

// State of the one-launch triangular solve: per-block flags tagged with a
// call epoch and a ticket counter that hands out blocks in dispatch order.
struct TrsvState {
  uint32_t* flags;     // device, max_blocks entries
  uint64_t* ticket;    // device counter, only ever incremented
  int32_t* err;        // device, set when a bounded wait expires (1) or tickets are out of step (2)
  int32_t* sing;       // device, set by getrs when a diagonal entry of U is exactly zero
  int64_t max_blocks;  // capacity of flags: ceil(rows / 64) (128-row blocks use half)
  uint32_t epoch;      // host copy of the last epoch used
  uint64_t tickets;    // host copy of the tickets handed out so far
};

// x := L^{-1} x (unit lower, lower = true) or U^{-1} x (non-unit upper) for
// one right-hand side, with L/U in the n x n matrix A.
template <typename T>
hipError_t trsv_wave(hipStream_t s, bool lower, int64_t n, const T* A, int64_t lda, T* x, TrsvState* st);

// *flag = 1 when some A(k,k), k < n, is exactly zero (flag untouched otherwise).
template <typename T>
hipError_t diag_zero_check(hipStream_t s, int64_t n, const T* A, int64_t lda, int32_t* flag);

// r = b - A x in FP64 (deterministic: nchunk column chunks, part holds nchunk*n)
hipError_t residual(hipStream_t s, int64_t n, const double* A, int64_t lda, const double* x, const double* b,
                    double* r, double* part, int64_t nchunk);
// *out = max(*out, max_i |v_i|) as the bit pattern of a double (*out starts at 0)
hipError_t absmax(hipStream_t s, int64_t n, const double* v, unsigned long long* out);
// *out = max(*out, ||A||_inf) (part holds nchunk*n)
hipError_t norm_inf_mat(hipStream_t s, int64_t n, const double* A, int64_t lda, double* part, int64_t nchunk,
                        unsigned long long* out);
hipError_t d2s_mat(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst,
                   int64_t ldd);
hipError_t d2s_vec(hipStream_t s, int64_t n, const double* src, float* dst);
// y = x + alpha * z
hipError_t axpy_s2d(hipStream_t s, int64_t n, double alpha, const float* z, const double* x, double* y);
// y = alpha * z
hipError_t s2d_scaled(hipStream_t s, int64_t n, double alpha, const float* z, double* y);
// out[c] = V(:, c) . w for c < k (k <= 64); part holds ceil(n/256)*k
hipError_t mdot(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* part,
                double* out);
// w -= V(:, 0:k) h
hipError_t mgemv_sub(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w);
// y += V(:, 0:k) c
hipError_t mgemv_add(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* c, double* y);
// dst = alpha * src
hipError_t scale_copy(hipStream_t s, int64_t n, double alpha, const double* src, double* dst);
// x += d
hipError_t vec_add(hipStream_t s, int64_t n, const double* d, double* x);
// dst[i] = (float)(src[perm[i]] / *smax)   (*smax: bit pattern of a double >= 0)
hipError_t gather_scale(hipStream_t s, int64_t n, const int32_t* perm, const double* src,
                        const unsigned long long* smax, float* dst);
// y = x + sign * (*smax) * z   (x may be NULL for zero, or equal to y)
hipError_t axpy_dev(hipStream_t s, int64_t n, double sign, const unsigned long long* smax, const float* z,
                    const double* x, double* y);

hipError_t set_int(hipStream_t s, int32_t* p, int32_t v);
hipError_t reset_flags(hipStream_t s, LeafSlots* ws);

}  // namespace lupp
