// Row interchanges (laswp) and the small triangular-solve leaf.
//
// laswp applies a step's sequential interchanges to the columns outside the
// column block (the paper's in-place, right-looking update order, Section 3.2:
// the current factor is overwritten at every step).  The run of interchanges
// is first composed into one permutation of the rows it touches (a single
// wavefront replays the swaps on row labels in LDS), then every (row, column)
// element moves once, in parallel: reads of a band of columns, a barrier,
// writes.  A swap chain never becomes a per-thread chain of dependent memory
// accesses.
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

// One wavefront replays interchanges k1..k2-1 on row labels.  Rows k1..k2-1
// are tracked in s_cont; rows below k2 that are hit are appended to a short
// list and found again by a ballot over it.
__global__ __launch_bounds__(64) void k_swap_pairs(const int32_t* __restrict__ ipiv, int64_t k1, int64_t k2,
                                                   int64_t m, SwapPairs* __restrict__ out) {
  __shared__ int32_t s_piv[kMaxSwaps];
  __shared__ int32_t s_cont[kMaxSwaps];
  __shared__ int32_t s_erow[kMaxSwaps];
  __shared__ int32_t s_econt[kMaxSwaps];
  const int lane = threadIdx.x;
  const int S = (int)(k2 - k1);
  for (int i = lane; i < S; i += 64) {
    s_piv[i] = ipiv[k1 + i] - 1;
    s_cont[i] = (int32_t)(k1 + i);
  }
  __syncthreads();
  int n_ext = 0;
  for (int i = 0; i < S; ++i) {
    const int64_t p = s_piv[i];
    const int64_t row = k1 + i;
    if (p <= row || p >= m) continue;  // no interchange (or NaN-born index)
    if (p < k2) {
      if (lane == 0) {
        const int32_t t = s_cont[i];
        s_cont[i] = s_cont[p - k1];
        s_cont[p - k1] = t;
      }
    } else {
      int found = -1;
      for (int e0 = 0; e0 < n_ext; e0 += 64) {
        const int e = e0 + lane;
        const unsigned long long hit = __ballot(e < n_ext && s_erow[e] == (int32_t)p);
        if (hit) {
          found = e0 + __ffsll((long long)hit) - 1;
          break;
        }
      }
      if (found < 0) {
        found = n_ext++;
        if (lane == 0) {
          s_erow[found] = (int32_t)p;
          s_econt[found] = (int32_t)p;
        }
      }
      if (lane == 0) {
        const int32_t t = s_cont[i];
        s_cont[i] = s_econt[found];
        s_econt[found] = t;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // lane 0's LDS writes precede the next replay step
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = lane; i < S; i += 64) {
    out->dst[i] = (int32_t)(k1 + i);
    out->src[i] = s_cont[i];
  }
  for (int e = lane; e < n_ext; e += 64) {
    out->dst[S + e] = s_erow[e];
    out->src[S + e] = s_econt[e];
  }
  if (lane == 0) out->count = S + n_ext;
}

// Gather/scatter of a composed row permutation on a band of 64 columns per
// workgroup, 8 columns at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_pairs(T* __restrict__ A, int64_t lda, int64_t c0, int64_t c1,
                                                     int64_t skip0, int64_t skip1,
                                                     const SwapPairs* __restrict__ pairs) {
  constexpr int CB = 64, CC = 8, QP = (2 * kMaxSwaps) / 256;
  __shared__ int32_t s_dst[2 * kMaxSwaps];
  __shared__ int32_t s_src[2 * kMaxSwaps];
  const int tid = threadIdx.x;
  const int P = pairs->count;
  for (int q = tid; q < P; q += 256) {
    s_dst[q] = pairs->dst[q];
    s_src[q] = pairs->src[q];
  }
  __syncthreads();
  const int64_t width = (c1 - c0) - (skip1 - skip0);
  const int64_t t0 = (int64_t)blockIdx.x * CB;
  for (int cc0 = 0; cc0 < CB; cc0 += CC) {
    T v[QP][CC];
#pragma unroll
    for (int qi = 0; qi < QP; ++qi) {
      const int q = tid + 256 * qi;
#pragma unroll
      for (int cc = 0; cc < CC; ++cc) {
        const int64_t t = t0 + cc0 + cc;
        int64_t c = c0 + t;
        if (c >= skip0) c += (skip1 - skip0);
        if (q < P && t < width) v[qi][cc] = A[(int64_t)s_src[q] + c * lda];
      }
    }
    __syncthreads();
#pragma unroll
    for (int qi = 0; qi < QP; ++qi) {
      const int q = tid + 256 * qi;
#pragma unroll
      for (int cc = 0; cc < CC; ++cc) {
        const int64_t t = t0 + cc0 + cc;
        int64_t c = c0 + t;
        if (c >= skip0) c += (skip1 - skip0);
        if (q < P && t < width) A[(int64_t)s_dst[q] + c * lda] = v[qi][cc];
      }
    }
    __syncthreads();
  }
}

// One thread per right-hand column, the triangle in LDS (read as broadcasts),
// no barrier inside the substitution.  The column is solved in chunks of 16
// rows: a chunk lives in registers, finished rows in LDS (each lane its own
// column, so lanes touch consecutive LDS words).
template <typename T, bool LOWER>
__global__ __launch_bounds__(64) void k_trsm_small(int w, int64_t ncols, const T* __restrict__ L, int64_t ldl,
                                                   T* __restrict__ B, int64_t ldb) {
  constexpr int WM = 64, CH = 16;
  __shared__ T sL[WM * WM];  // sL[kk * WM + i] = L(i, kk)
  __shared__ T sX[WM * 64];  // sX[i * 64 + lane] = row i of this lane's column
  const int tid = threadIdx.x;
  for (int e = tid; e < WM * WM; e += 64) {
    const int i = e % WM, kk = e / WM;
    sL[e] = (i < w && kk < w) ? L[i + (int64_t)kk * ldl] : T(0);
  }
  const int64_t c = (int64_t)blockIdx.x * 64 + tid;
  const bool active = c < ncols;
  T* col = B + (active ? c : 0) * ldb;
  for (int i = 0; i < WM; ++i) sX[i * 64 + tid] = (active && i < w) ? col[i] : T(0);
  __syncthreads();
  const int nch = (w + CH - 1) / CH;
  for (int q = 0; q < nch; ++q) {
    const int ch = LOWER ? q : (nch - 1 - q);
    const int r0 = ch * CH;
    T x[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) x[i] = sX[(r0 + i) * 64 + tid];
    if (LOWER) {
      for (int kk = 0; kk < r0; ++kk) {  // finished rows above the chunk
        const T xk = sX[kk * 64 + tid];
#pragma unroll
        for (int i = 0; i < CH; ++i) x[i] = x[i] - sL[kk * WM + r0 + i] * xk;
      }
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) {
        const T xk = x[kk];
#pragma unroll
        for (int i = kk + 1; i < CH; ++i) x[i] = x[i] - sL[(r0 + kk) * WM + r0 + i] * xk;
      }
    } else {
      for (int kk = r0 + CH; kk < w; ++kk) {  // finished rows below the chunk
        const T xk = sX[kk * 64 + tid];
#pragma unroll
        for (int i = 0; i < CH; ++i) x[i] = x[i] - sL[kk * WM + r0 + i] * xk;
      }
#pragma unroll
      for (int kk = CH - 1; kk >= 0; --kk) {
        if (r0 + kk < w) x[kk] = x[kk] / sL[(r0 + kk) * WM + r0 + kk];
        const T xk = x[kk];
#pragma unroll
        for (int i = 0; i < kk; ++i) x[i] = x[i] - sL[(r0 + kk) * WM + r0 + i] * xk;
      }
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) sX[(r0 + i) * 64 + tid] = x[i];
  }
  if (active)
    for (int i = 0; i < w; ++i) col[i] = sX[i * 64 + tid];
}

__global__ void k_set_int(int32_t* p, int32_t v) { *p = v; }

}  // namespace

hipError_t swap_pairs(hipStream_t s, const int32_t* ipiv, int64_t k1, int64_t k2, int64_t m, SwapPairs* pairs) {
  if (k2 - k1 > kMaxSwaps || k2 < k1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_swap_pairs, dim3(1), dim3(64), 0, s, ipiv, k1, k2, m, pairs);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_pairs(hipStream_t s, T* A, int64_t lda, int64_t c0, int64_t c1, int64_t skip0, int64_t skip1,
                       const SwapPairs* pairs, int64_t max_pairs) {
  (void)max_pairs;
  if (skip0 < c0) skip0 = c0;
  if (skip1 > c1) skip1 = c1;
  if (skip1 < skip0) skip1 = skip0;
  const int64_t width = (c1 - c0) - (skip1 - skip0);
  if (width <= 0) return hipSuccess;
  const int64_t blocks = (width + 63) / 64;
  hipLaunchKernelGGL(k_apply_pairs<T>, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, c0, c1, skip0, skip1, pairs);
  return hipGetLastError();
}

template <typename T>
hipError_t laswp(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t c0, int64_t c1, int64_t skip0, int64_t skip1,
                 const int32_t* ipiv, int64_t k1, int64_t k2, SwapPairs* pairs) {
  if (skip0 < c0) skip0 = c0;
  if (skip1 > c1) skip1 = c1;
  if (skip1 < skip0) skip1 = skip0;
  const int64_t width = (c1 - c0) - (skip1 - skip0);
  if (width <= 0 || k2 <= k1) return hipSuccess;
  if (pairs && k2 - k1 <= kMaxSwaps) {
    hipError_t e = swap_pairs(s, ipiv, k1, k2, m, pairs);
    if (e != hipSuccess) return e;
    return apply_pairs<T>(s, A, lda, c0, c1, skip0, skip1, pairs, 2 * (k2 - k1));
  }
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

template <typename T>
hipError_t trsm_small(hipStream_t s, bool lower, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B,
                      int64_t ldb) {
  if (w <= 0 || ncols <= 0) return hipSuccess;
  if (w > 64) return hipErrorInvalidValue;
  const int64_t blocks = (ncols + 63) / 64;
  if (lower)
    hipLaunchKernelGGL((k_trsm_small<T, true>), dim3((unsigned)blocks), dim3(64), 0, s, (int)w, ncols, L, ldl, B, ldb);
  else
    hipLaunchKernelGGL((k_trsm_small<T, false>), dim3((unsigned)blocks), dim3(64), 0, s, (int)w, ncols, L, ldl, B,
                       ldb);
  return hipGetLastError();
}

template hipError_t trsm_small<double>(hipStream_t, bool, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template hipError_t trsm_small<float>(hipStream_t, bool, int64_t, int64_t, const float*, int64_t, float*, int64_t);

hipError_t set_int(hipStream_t s, int32_t* p, int32_t v) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

template hipError_t laswp<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                  const int32_t*, int64_t, int64_t, SwapPairs*);
template hipError_t laswp<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                 const int32_t*, int64_t, int64_t, SwapPairs*);
template hipError_t apply_pairs<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        const SwapPairs*, int64_t);
template hipError_t apply_pairs<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                       const SwapPairs*, int64_t);
template hipError_t trsm_leaf<double>(hipStream_t, bool, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template hipError_t trsm_leaf<float>(hipStream_t, bool, int64_t, int64_t, const float*, int64_t, float*, int64_t);

}  // namespace lupp
