// Triangular solve with the unit lower triangle of a column block (order
// w <= 256) for many right-hand columns in one launch: U12 := inv(L11) * A12
// of the right-looking step (the paper's TRSM, Section 3.2), and the same
// inside the recursive column-block factorization.
#include "common.h"
#include "wave.h"

namespace lupp {
namespace {

// B := inv(L) * B for a unit lower triangle of order w <= 256, one launch.
// Lane (r, grp) of a wavefront holds rows r, r+16, ..., r+240 of CPT
// right-hand columns in registers; a workgroup covers 4 waves x 4 groups x
// CPT columns.  The triangle is consumed in 16-column chunks staged through
// LDS (double-buffered: the next chunk's loads are in flight while the current
// one is applied).  Within a chunk, step k broadcasts row 16q+k (final at that
// point) from lane k of each 16-lane row and subtracts its multiple from every
// row below it, the chunk's own rows and all later ones, so each row
// accumulates b_i - sum_j l_ij x_j in increasing j, as plain forward
// substitution does.
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_trsm_lower_band(int w, int64_t ncols, const T* __restrict__ L, int64_t ldl,
                                                         T* __restrict__ B, int64_t ldb) {
  constexpr int CH = 16, MAXW = kTrsmBandMaxW, NQ = MAXW / CH;
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
  const int nq = (w + CH - 1) / CH;
  T pf[CH];
  auto load_panel = [&](int q) {
    const int j0 = q * CH;
#pragma unroll
    for (int kk = 0; kk < CH; ++kk) {
      const int j = j0 + kk;
      pf[kk] = (tid >= j0 && tid < w && j < w) ? L[tid + (int64_t)j * ldl] : T(0);
    }
  };
  auto store_panel = [&](int b) {
#pragma unroll
    for (int kk = 0; kk < CH; ++kk) sL[b][kk][tid] = pf[kk];
  };
  load_panel(0);
  store_panel(0);
  __syncthreads();
  static_for<0, NQ>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    if (q < nq) {
      constexpr int b = q & 1;
      if (q + 1 < nq) load_panel(q + 1);
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
          if (t < nq) {
            const T l = sL[b][k][t * CH + r];
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) x[t][cc] = x[t][cc] - l * bv[cc];
          }
        }
      });
      if (q + 1 < nq) store_panel(b ^ 1);
      __syncthreads();
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

}  // namespace

template <typename T>
hipError_t trsm_lower_band(hipStream_t s, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B, int64_t ldb) {
  if (w <= 0 || ncols <= 0) return hipSuccess;
  if (w > kTrsmBandMaxW) return hipErrorInvalidValue;
  // a workgroup covers 16 * CPT columns; four per thread once that still
  // leaves a few hundred workgroups
  if (ncols >= 128 * 64) {
    const int64_t blocks = (ncols + 63) / 64;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_trsm_lower_band<T, 4>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl, B,
                       ldb);
  } else {
    const int64_t blocks = (ncols + 15) / 16;
    hipLaunchKernelGGL((k_trsm_lower_band<T, 1>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl, B,
                       ldb);
  }
  return hipGetLastError();
}

template hipError_t trsm_lower_band<double>(hipStream_t, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template hipError_t trsm_lower_band<float>(hipStream_t, int64_t, int64_t, const float*, int64_t, float*, int64_t);

}  // namespace lupp
