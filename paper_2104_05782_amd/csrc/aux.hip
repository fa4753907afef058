// Row interchanges (laswp) and the small triangular-solve leaf.
//
// laswp applies a step's sequential interchanges to the columns outside the
// column block (the paper's in-place, right-looking update order, Section 3.2:
// the current factor is overwritten at every step).  Column-major storage puts
// the two elements of a swap in the same column, so one thread owns one
// column and performs the interchanges in order; the pivots are staged once
// per workgroup in LDS.
//
// trsm_leaf solves with a w x w triangle (w <= 64) for a band of 64 right-hand
// columns per workgroup, entirely in LDS: U12 := inv(L11) * A12 (unit lower,
// forward) inside the factorization and the back substitution with U in the
// solve.  Larger triangles are split recursively by the host around the GEMM.
#include "common.h"

namespace lupp {
namespace {

constexpr int kSwapChunk = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_laswp(T* __restrict__ A, int64_t lda, int64_t c0, int64_t c1,
                                               int64_t skip0, int64_t skip1, const int32_t* __restrict__ ipiv,
                                               int64_t k1, int64_t k2, int64_t nrows) {
  __shared__ int32_t s_piv[kSwapChunk];
  const int64_t width = (c1 - c0) - (skip1 - skip0);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = c0 + t;
  if (c >= skip0) c += (skip1 - skip0);
  const bool active = t < width;
  T* col = A + c * lda;
  for (int64_t kb = k1; kb < k2; kb += kSwapChunk) {
    const int64_t kn = min((int64_t)kSwapChunk, k2 - kb);
    __syncthreads();
    if (threadIdx.x < kn) s_piv[threadIdx.x] = ipiv[kb + threadIdx.x];
    __syncthreads();
    if (active) {
      for (int64_t q = 0; q < kn; ++q) {
        const int64_t i = kb + q;
        const int64_t p = (int64_t)s_piv[q] - 1;
        if (p != i && p >= 0 && p < nrows) {
          const T x = col[i];
          col[i] = col[p];
          col[p] = x;
        }
      }
    }
  }
}

template <typename T, bool LOWER>
__global__ __launch_bounds__(256) void k_trsm_leaf(int w, int64_t ncols, const T* __restrict__ L, int64_t ldl,
                                                   T* __restrict__ B, int64_t ldb) {
  __shared__ T sL[64][65];
  __shared__ T sB[64][64];
  const int tid = threadIdx.x;
  const int c = tid & 63, rg = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < w * w; e += 256) {
    const int i = e % w, kk = e / w;
    sL[i][kk] = L[i + (int64_t)kk * ldl];
  }
  for (int e = tid; e < w * 64; e += 256) {
    const int i = e % w, cc = e / w;
    const int64_t gc = c0 + cc;
    sB[i][cc] = (gc < ncols) ? B[i + gc * ldb] : T(0);
  }
  if (LOWER) {
    for (int kk = 0; kk < w; ++kk) {
      __syncthreads();
      const T x = sB[kk][c];
      for (int i = kk + 1 + rg; i < w; i += 4) sB[i][c] = sB[i][c] - sL[i][kk] * x;
    }
  } else {
    for (int kk = w - 1; kk >= 0; --kk) {
      __syncthreads();
      if (rg == 0) sB[kk][c] = sB[kk][c] / sL[kk][kk];
      __syncthreads();
      const T x = sB[kk][c];
      for (int i = rg; i < kk; i += 4) sB[i][c] = sB[i][c] - sL[i][kk] * x;
    }
  }
  __syncthreads();
  for (int e = tid; e < w * 64; e += 256) {
    const int i = e % w, cc = e / w;
    const int64_t gc = c0 + cc;
    if (gc < ncols) B[i + gc * ldb] = sB[i][cc];
  }
}

__global__ void k_set_int(int32_t* p, int32_t v) { *p = v; }

}  // namespace

template <typename T>
hipError_t laswp(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t c0, int64_t c1, int64_t skip0, int64_t skip1,
                 const int32_t* ipiv, int64_t k1, int64_t k2) {
  if (skip0 < c0) skip0 = c0;
  if (skip1 > c1) skip1 = c1;
  if (skip1 < skip0) skip1 = skip0;
  const int64_t width = (c1 - c0) - (skip1 - skip0);
  if (width <= 0 || k2 <= k1) return hipSuccess;
  const int64_t blocks = (width + 255) / 256;
  // an interchange outside rows [0, m) is ignored (it can only come from NaN input)
  hipLaunchKernelGGL(k_laswp<T>, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, c0, c1, skip0, skip1, ipiv, k1,
                     k2, m);
  return hipGetLastError();
}

template <typename T>
hipError_t trsm_leaf(hipStream_t s, bool lower, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B,
                     int64_t ldb) {
  if (w <= 0 || ncols <= 0) return hipSuccess;
  if (w > 64) return hipErrorInvalidValue;
  const int64_t blocks = (ncols + 63) / 64;
  if (lower)
    hipLaunchKernelGGL((k_trsm_leaf<T, true>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl, B, ldb);
  else
    hipLaunchKernelGGL((k_trsm_leaf<T, false>), dim3((unsigned)blocks), dim3(256), 0, s, (int)w, ncols, L, ldl, B,
                       ldb);
  return hipGetLastError();
}

hipError_t set_int(hipStream_t s, int32_t* p, int32_t v) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

template hipError_t laswp<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                  const int32_t*, int64_t, int64_t);
template hipError_t laswp<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                 const int32_t*, int64_t, int64_t);
template hipError_t trsm_leaf<double>(hipStream_t, bool, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template hipError_t trsm_leaf<float>(hipStream_t, bool, int64_t, int64_t, const float*, int64_t, float*, int64_t);

}  // namespace lupp
