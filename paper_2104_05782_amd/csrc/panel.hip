// Column-block ("panel") factorization with partial pivoting: the leaf of the
// recursive panel.  The paper singles this step out as the one that limits a
// blocked LU: it works on few data and every other step waits for it
// (Section 4.1).  Its latency is a chain of w dependent pivot decisions, each
// a reduction over all r rows of the block.
//
// Design (gfx950): G workgroups of 256 threads split the r rows; every thread
// keeps RPT rows x W columns of the block in registers for the whole call, so
// the rank-1 updates never touch memory.  Per column j:
//   1. each thread scans its rows, wavefront shuffles and LDS reduce to the
//      workgroup's best (|a|, row) under the total order (|a| desc, row asc):
//      any reduction tree then reproduces the sequential first-maximum scan;
//   2. with G > 1 each workgroup publishes its candidate and the candidate's
//      row (and the owner of row j publishes row j) to its own slot, then
//      raises its own progress flag; every workgroup polls all G flags (no
//      shared counter, so no atomic contention) and reduces the G candidates;
//   3. interchange (the two owning threads exchange whole rows), true-division
//      scaling of column j, rank-1 update of the remaining columns.
// Wait loops are bounded: an expired wait sets ws->err and the kernel finishes.
#include "common.h"

namespace lupp {
namespace {

constexpr int NT = 256;
constexpr long kSpinLimit = 1L << 22;

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void st_u64(void* p, uint64_t v) {
  __hip_atomic_store((uint64_t*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_u64(const void* p) {
  return __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f64(double* p, double v) { st_u64(p, __double_as_longlong(v)); }
__device__ __forceinline__ double ld_f64(const double* p) { return __longlong_as_double(ld_u64(p)); }

template <typename T, int W, int RPT>
__global__ __launch_bounds__(NT) void k_panel_leaf(int64_t r, int w, T* __restrict__ P, int64_t ld,
                                                   int32_t* __restrict__ ipiv, int64_t k,
                                                   int32_t* __restrict__ info, LeafSlots* __restrict__ ws,
                                                   uint32_t epoch) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int64_t rbase = (int64_t)g * NT * RPT;

  __shared__ T s_prow[W];
  __shared__ T s_rowj[W];
  __shared__ double s_wv[NT / 64];
  __shared__ int64_t s_wi[NT / 64];
  __shared__ double s_bv;
  __shared__ int64_t s_bi;
  __shared__ int s_broken;

  T a[RPT][W];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = rbase + q * NT + tid;
#pragma unroll
    for (int c = 0; c < W; ++c) a[q][c] = (i < r && c < w) ? P[i + c * ld] : T(0);
  }
  if (tid == 0) s_broken = 0;
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    const int par = j & 1;
    // 1. local candidate
    double bv = -1.0;
    int64_t bi = INT64_MAX;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t i = rbase + q * NT + tid;
      T x = T(0);
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c == j) x = a[q][c];
      const double v = fabs((double)x);
      if (i >= j && i < r && better(v, i, bv, bi)) {
        bv = v;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int64_t oi = __shfl_xor(bi, off);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_wv[wave] = bv;
      s_wi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = s_wv[0];
      int64_t i = s_wi[0];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q)
        if (better(s_wv[q], s_wi[q], v, i)) {
          v = s_wv[q];
          i = s_wi[q];
        }
      s_bv = v;
      s_bi = i;
    }
    __syncthreads();
    const int64_t wg_best = s_bi;

    // 2. publish and combine
    if (G == 1) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        if (i == wg_best) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_prow[c] = a[q][c];
        }
        if (i == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_rowj[c] = a[q][c];
        }
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        if (i == wg_best && wg_best < r) {
#pragma unroll
          for (int c = 0; c < W; ++c) st_f64(&ws->cand_row[par][g][c], (double)a[q][c]);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        if (i == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) st_f64(&ws->rowj[par][c], (double)a[q][c]);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
      }
      if (tid == 0) {
        st_f64(&ws->cand_val[par][g], s_bv);
        st_u64(&ws->cand_idx[par][g], (uint64_t)s_bi);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      }
      __syncthreads();
      const uint32_t target = epoch + (uint32_t)j + 1u;
      if (tid == 0) __hip_atomic_store(&ws->flags[g], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (wave == 0) {
        if (!s_broken) {
          long spins = 0;
          for (;;) {
            bool ok = true;
            for (int q = lane; q < G; q += 64)
              ok &= __hip_atomic_load(&ws->flags[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
            if (__all(ok)) break;
            if (++spins > kSpinLimit) {
              if (lane == 0) {
                __hip_atomic_store(&ws->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_broken = 1;
              }
              break;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double v = -1.0;
        int64_t i = INT64_MAX;
        int gw = 0;
        for (int q = lane; q < G; q += 64) {
          const double qv = ld_f64(&ws->cand_val[par][q]);
          const int64_t qi = (int64_t)ld_u64(&ws->cand_idx[par][q]);
          if (better(qv, qi, v, i)) {
            v = qv;
            i = qi;
            gw = q;
          }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          const double ov = __shfl_xor(v, off);
          const int64_t oi = __shfl_xor(i, off);
          const int og = __shfl_xor(gw, off);
          if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
            gw = og;
          }
        }
        if (lane < W) {
          s_prow[lane] = (T)ld_f64(&ws->cand_row[par][gw][lane]);
          s_rowj[lane] = (T)ld_f64(&ws->rowj[par][lane]);
        }
        if (lane == 0) s_bi = i;
      }
      __syncthreads();
    }

    // 3. interchange, scale, update (a winner outside the block can only come
    // from NaN input: keep the diagonal row then)
    int64_t piv = s_bi;
    if (piv < j || piv >= r) piv = j;
    const T pv = s_prow[j];
    if (g == 0 && tid == 0) {
      ipiv[k + j] = (int32_t)(k + piv + 1);
      if (pv == T(0) && *info == 0) *info = (int32_t)(k + j + 1);
    }
    if (pv != T(0)) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        if (i == piv && piv != j) {
#pragma unroll
          for (int c = 0; c < W; ++c) a[q][c] = s_rowj[c];
        } else if (i == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) a[q][c] = s_prow[c];
        }
        if (i > j && i < r) {
          T x = T(0);
#pragma unroll
          for (int c = 0; c < W; ++c)
            if (c == j) x = a[q][c];
          const T l = x / pv;
#pragma unroll
          for (int c = 0; c < W; ++c) {
            if (c == j) a[q][c] = l;
            if (c > j) a[q][c] = a[q][c] - l * s_prow[c];
          }
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = rbase + q * NT + tid;
    if (i < r) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < w) P[i + c * ld] = a[q][c];
    }
  }
}

__global__ void k_reset_flags(LeafSlots* ws) {
  for (int i = threadIdx.x; i < kLeafMaxGroups; i += blockDim.x) ws->flags[i] = 0;
}

template <typename T, int W, int RPT>
hipError_t launch_leaf(hipStream_t s, int G, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k,
                       int32_t* info, LeafSlots* ws, uint32_t epoch) {
  hipLaunchKernelGGL((k_panel_leaf<T, W, RPT>), dim3(G), dim3(NT), 0, s, r, w, P, ld, ipiv, k, info, ws, epoch);
  return hipGetLastError();
}

}  // namespace

hipError_t reset_flags(hipStream_t s, LeafSlots* ws) {
  hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(256), 0, s, ws);
  return hipGetLastError();
}

template <typename T>
hipError_t panel_leaf(hipStream_t s, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k, int32_t* info,
                      LeafSlots* ws, uint32_t epoch) {
  if (w <= 0 || r <= 0) return hipSuccess;
  if (w > kLeafMaxWidth) return hipErrorInvalidValue;
  // rows per thread: fewest workgroups (cheapest exchange) that keep the
  // block in registers
  int rpt;
  if (r <= NT * 4) rpt = (r <= NT) ? 1 : (r <= 2 * NT ? 2 : 4);
  else rpt = (r <= (int64_t)16 * NT * 2) ? 2 : 4;
  const int64_t G64 = (r + (int64_t)NT * rpt - 1) / ((int64_t)NT * rpt);
  if (G64 > kLeafMaxGroups) return hipErrorInvalidValue;
  const int G = (int)G64;
  if (w <= 16) {
    if (rpt == 1) return launch_leaf<T, 16, 1>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
    if (rpt == 2) return launch_leaf<T, 16, 2>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
    return launch_leaf<T, 16, 4>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
  }
  if (rpt == 1) return launch_leaf<T, 32, 1>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
  if (rpt == 2) return launch_leaf<T, 32, 2>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
  return launch_leaf<T, 32, 4>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch);
}

template hipError_t panel_leaf<double>(hipStream_t, int64_t, int, double*, int64_t, int32_t*, int64_t, int32_t*,
                                       LeafSlots*, uint32_t);
template hipError_t panel_leaf<float>(hipStream_t, int64_t, int, float*, int64_t, int32_t*, int64_t, int32_t*,
                                      LeafSlots*, uint32_t);

}  // namespace lupp
