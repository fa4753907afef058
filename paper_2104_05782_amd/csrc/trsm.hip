// Triangular solve with the unit lower triangle of a column block (order
// w <= 256) for many right-hand columns in one launch: U12 := inv(L11) * A12
// of the right-looking step (the paper's TRSM, Section 3.2), and the same
// inside the recursive column-block factorization.
#include "common.h"
#include "wave.h"

namespace lupp {
namespace {

// B := inv(L) * B for a unit lower triangle of order w <= 16 NQ (NQ <= 16),
// one launch.  Lane (r, grp) of a wavefront holds rows r, r+16, ..., r+16(NQ-1)
// of CPT right-hand columns in registers; a workgroup covers 4 waves x 4
// groups x CPT columns.  The triangle is consumed in 16-column chunks staged through
// LDS (double-buffered: the next chunk's loads are in flight while the current
// one is applied).  Within a chunk, step k broadcasts row 16q+k (final at that
// point) from lane k of each 16-lane row and subtracts its multiple from every
// row below it, the chunk's own rows and all later ones, so each row
// accumulates b_i - sum_j l_ij x_j in increasing j, as plain forward
// substitution does.  The later chunks are updated without a per-chunk test
// of w (a runtime branch there serializes each update's LDS read): rows at or
// past w hold zeros of L in LDS and are never stored.
template <typename T, int CPT, int NQ>
__global__ __launch_bounds__(256) void k_trsm_lower_band(int w, int64_t ncols, const T* __restrict__ L, int64_t ldl,
                                                         T* __restrict__ B, int64_t ldb) {
  constexpr int CH = 16, MAXW = NQ * CH;
  static_assert(NQ >= 1 && MAXW <= kTrsmBandMaxW, "band order");
  constexpr int NC = 4 * CPT;  // columns per wavefront (four 16-lane groups)
  __shared__ T sL[2][CH][MAXW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, grp = lane >> 4;
  const int64_t cb = (int64_t)blockIdx.x * (4 * NC) + wave * NC + grp * CPT;
  T x[NQ][CPT];
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    const int i = t * CH + r;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int64_t c = cb + cc;
      x[t][cc] = (i < w && c < ncols) ? B[i + c * ldb] : T(0);
    }
  }
  T pf[CH];
  // (the address is clamped into the triangle, so the load needs no branch)
  const int rl = tid < w ? tid : w - 1;
  auto load_panel = [&](int q) {
    const int j0 = q * CH;
#pragma unroll
    for (int kk = 0; kk < CH; ++kk) {
      const int j = j0 + kk;
      const T v = L[rl + (int64_t)(j < w ? j : w - 1) * ldl];
      pf[kk] = (tid >= j0 && tid < w && j < w) ? v : T(0);
    }
  };
  auto store_panel = [&](int b) {
    if (tid < MAXW) {
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) sL[b][kk][tid] = pf[kk];
    }
  };
  load_panel(0);
  store_panel(0);
  __syncthreads();
  static_for<0, NQ>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    {
      constexpr int b = q & 1;
      if constexpr (q + 1 < NQ) load_panel(q + 1);
      static_for<0, CH>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        T bv[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) bv[cc] = row_bcast<k>(x[q][cc]);
        const T lq = sL[b][k][q * CH + r];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
          const T nv = x[q][cc] - lq * bv[cc];
          x[q][cc] = (r > k) ? nv : x[q][cc];
        }
#pragma unroll
        for (int t = q + 1; t < NQ; ++t) {
          const T l = sL[b][k][t * CH + r];
#pragma unroll
          for (int cc = 0; cc < CPT; ++cc) x[t][cc] = x[t][cc] - l * bv[cc];
        }
        // each step's updates are done in the step (moved later, their
        // operands would stay live and exhaust the registers)
#pragma unroll
        for (int t = q; t < NQ; ++t)
#pragma unroll
          for (int cc = 0; cc < CPT; ++cc) asm volatile("" : "+v"(x[t][cc]));
      });
      if constexpr (q + 1 < NQ) {
        store_panel(b ^ 1);
        __syncthreads();
      }
    }
  });
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    const int i = t * CH + r;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int64_t c = cb + cc;
      if (i < w && c < ncols) B[i + c * ldb] = x[t][cc];
    }
  }
}

template <typename T, int NQ>
void launch_band(hipStream_t s, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B, int64_t ldb,
                 int64_t blocks, bool wide) {
  if (wide)
    hipLaunchKernelGGL((k_trsm_lower_band<T, 4, NQ>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl,
                       B, ldb);
  else
    hipLaunchKernelGGL((k_trsm_lower_band<T, 1, NQ>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl,
                       B, ldb);
}

}  // namespace

template <typename T>
hipError_t trsm_lower_band(hipStream_t s, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B, int64_t ldb) {
  if (w <= 0 || ncols <= 0) return hipSuccess;
  if (w > kTrsmBandMaxW) return hipErrorInvalidValue;
  // a workgroup covers 16 * CPT columns; four per thread once that still
  // leaves a few hundred workgroups
  const bool wide = ncols >= 128 * 64;
  const int64_t blocks = wide ? (ncols + 63) / 64 : (ncols + 15) / 16;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  // row chunks held per lane: the order rounded up to 64, 128 or 256
  if (w <= 64)
    launch_band<T, 4>(s, w, ncols, L, ldl, B, ldb, blocks, wide);
  else if (w <= 128)
    launch_band<T, 8>(s, w, ncols, L, ldl, B, ldb, blocks, wide);
  else
    launch_band<T, 16>(s, w, ncols, L, ldl, B, ldb, blocks, wide);
  return hipGetLastError();
}

template hipError_t trsm_lower_band<double>(hipStream_t, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template hipError_t trsm_lower_band<float>(hipStream_t, int64_t, int64_t, const float*, int64_t, float*, int64_t);

}  // namespace lupp
