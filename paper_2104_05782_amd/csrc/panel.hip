// Column-block ("panel") factorization with partial pivoting: the leaf of the
// recursive panel.  The paper singles this step out as the one that limits a
// blocked LU: it works on few data and every other step waits for it
// (Section 4.1).  Its latency is a chain of w dependent pivot decisions, each
// a reduction over all r rows of the block.
//
// Design (gfx950): G workgroups split the r rows; every thread keeps RPT rows
// x W columns of the block in registers for the whole call, so the rank-1
// updates never touch memory.  Per column j:
//   1. each thread scans its rows; wavefront shuffles and an LDS step reduce
//      to the workgroup's best (|a|, row) under the total order (|a| desc, row
//      asc), so any reduction tree reproduces the sequential first-maximum
//      scan;
//   2. with G > 1 each workgroup publishes its candidate, the candidate's row
//      (and, from the owner of row j, row j) with device-coherent stores,
//      waits for their completion, and raises its own progress flag; every
//      workgroup polls the G flags (no shared counter: no atomic contention),
//      then reads all G candidates and candidate rows in one round trip;
//   3. interchange (the two owning threads exchange whole rows), true-division
//      scaling of column j, rank-1 update of the remaining columns.
// The same interchange is applied to the other columns of the enclosing
// column block by threads that own one such column each; a step's loads are
// issued as soon as the pivot is known and its stores in the next step, so
// their latency hides behind the next pivot search.
// Wait loops are bounded: an expired wait sets ws->err and the kernel finishes.
#include "common.h"
#include "wave.h"

namespace lupp {
namespace {

constexpr long kSpinLimit = 1L << 22;
constexpr int kMaxOther = 4;  // other columns per thread

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

// wait until this thread's stores have completed (reached the coherence point)
__device__ __forceinline__ void drain_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Workgroup barrier that waits only for LDS traffic.  (__syncthreads also
// waits for every outstanding global load and store of the wave, which would
// put a memory round trip on each pivot step.)  The signal fences keep the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt untouched
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename T, int W, int RPT, int NT>
__global__ __launch_bounds__(NT) void k_panel_leaf(int64_t r, int w, T* __restrict__ P, int64_t ld,
                                                   int32_t* __restrict__ ipiv, int64_t k,
                                                   int32_t* __restrict__ info, LeafSlots* __restrict__ ws,
                                                   uint32_t epoch, int64_t oc_lo, int64_t oc_hi) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int64_t rbase = (int64_t)g * NT * RPT;

  __shared__ T s_prow[W];
  __shared__ T s_rowj[W];
  __shared__ double s_wv[2][NW];
  __shared__ int64_t s_wi[2][NW];
  __shared__ int64_t s_bi;
  __shared__ int s_broken;
  __shared__ int32_t s_ipiv[W];
  __shared__ int32_t s_zero;
  __shared__ double s_cv[kLeafMaxGroups];
  __shared__ int64_t s_ci[kLeafMaxGroups];
  __shared__ double s_crow[kLeafMaxGroups * W];

  T a[RPT][W];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = rbase + q * NT + tid;
#pragma unroll
    for (int c = 0; c < W; ++c) a[q][c] = (i < r && c < w) ? P[i + c * ld] : T(0);
  }

  // other columns of the enclosing block owned by this thread
  const int64_t n_left = -oc_lo, n_other = n_left + (oc_hi - w);
  const int64_t gt = (int64_t)g * NT + tid, gstride = (int64_t)G * NT;
  T* ocol[kMaxOther];
  bool own[kMaxOther];
#pragma unroll
  for (int u = 0; u < kMaxOther; ++u) {
    const int64_t q = gt + u * gstride;
    own[u] = q < n_other;
    const int64_t c = (q < n_left) ? (oc_lo + q) : (w + (q - n_left));
    ocol[u] = P + (own[u] ? c : 0) * ld;
  }
  bool pend = false;
  int64_t prj = 0, prp = 0;
  T pvj[kMaxOther], pvp[kMaxOther];

  if (tid == 0) {
    s_broken = 0;
    s_zero = 0;
  }
  __syncthreads();

  // fully unrolled over the W columns: every register index below is a
  // compile-time constant (no select chains over the row's registers)
#pragma clang loop unroll(full)
  for (int j = 0; j < W; ++j) {
    if (j < w) {
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
    wave_argmax(bv, bi);
    if (lane == 0) {
      s_wv[par][wave] = bv;
      s_wi[par][wave] = bi;
    }
    lds_barrier();
    // every thread combines the wavefront candidates itself (no extra barrier)
    double wg_v = s_wv[par][0];
    int64_t wg_best = s_wi[par][0];
#pragma unroll
    for (int q = 1; q < NW; ++q)
      if (better(s_wv[par][q], s_wi[par][q], wg_v, wg_best)) {
        wg_v = s_wv[par][q];
        wg_best = s_wi[par][q];
      }

    // 2. publish and combine
    int64_t gbest;
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
      lds_barrier();
      gbest = wg_best;
    } else {
      bool wrote = false;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        if (i == wg_best && wg_best < r) {
#pragma unroll
          for (int c = 0; c < W; ++c) st_f64(&ws->cand_row[par][g][c], (double)a[q][c]);
          wrote = true;
        }
        if (i == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) st_f64(&ws->rowj[par][c], (double)a[q][c]);
          wrote = true;
        }
      }
      if (tid == 0) {
        st_f64(&ws->cand_val[par][g], wg_v);
        st_u64(&ws->cand_idx[par][g], (uint64_t)wg_best);
        wrote = true;
      }
      if (wrote) drain_stores();
      lds_barrier();
      const uint32_t target = epoch + (uint32_t)j + 1u;
      if (wave == 0) {
        if (lane == 0) __hip_atomic_store(&ws->flags[g], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
      }
      lds_barrier();
      // one round trip: every candidate, every candidate row, row j
      for (int q = tid; q < G; q += NT) {
        s_cv[q] = ld_f64(&ws->cand_val[par][q]);
        s_ci[q] = (int64_t)ld_u64(&ws->cand_idx[par][q]);
      }
      for (int e = tid; e < G * W; e += NT) s_crow[e] = ld_f64(&ws->cand_row[par][e / W][e % W]);
      if (tid < W) s_rowj[tid] = (T)ld_f64(&ws->rowj[par][tid]);
      lds_barrier();
      if (wave == 0) {
        double v = -1.0;
        int64_t i = INT64_MAX;
        for (int q = lane; q < G; q += 64) {
          if (better(s_cv[q], s_ci[q], v, i)) {
            v = s_cv[q];
            i = s_ci[q];
          }
        }
        wave_argmax(v, i);
        // the winning row index identifies its workgroup
        const int gw = (i == INT64_MAX) ? 0 : (int)(i / ((int64_t)NT * RPT));
        if (lane < W) s_prow[lane] = (T)s_crow[gw * W + lane];
        if (lane == 0) s_bi = i;
      }
      lds_barrier();
      gbest = s_bi;
    }

    // 3. interchange, scale, update (a winner outside the block can only come
    // from NaN input: keep the diagonal row then)
    int64_t piv = gbest;
    if (piv < j || piv >= r) piv = j;
    const T pv = s_prow[j];
    if (tid == 0) {
      s_ipiv[j] = (int32_t)(k + piv + 1);
      if (pv == T(0) && s_zero == 0) s_zero = (int32_t)(k + j + 1);
    }
    // the same interchange on the other columns of the enclosing block:
    // stores of the previous step, loads of this one
    if (pend) {
#pragma unroll
      for (int u = 0; u < kMaxOther; ++u)
        if (own[u]) {
          ocol[u][prj] = pvp[u];
          ocol[u][prp] = pvj[u];
        }
      pend = false;
    }
    if (piv != j && pv != T(0)) {
#pragma unroll
      for (int u = 0; u < kMaxOther; ++u)
        if (own[u]) {
          pvj[u] = ocol[u][j];
          pvp[u] = ocol[u][piv];
        }
      pend = true;
      prj = j;
      prp = piv;
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
    // s_prow/s_rowj are rewritten only after the next column's first barrier,
    // which every wave reaches after finishing this column
    }
  }

  if (pend) {
#pragma unroll
    for (int u = 0; u < kMaxOther; ++u)
      if (own[u]) {
        ocol[u][prj] = pvp[u];
        ocol[u][prp] = pvj[u];
      }
  }
  lds_barrier();  // s_ipiv / s_zero complete
  if (g == 0) {
    for (int jj = tid; jj < w; jj += NT) ipiv[k + jj] = s_ipiv[jj];
    if (tid == 0 && s_zero != 0 && *info == 0) *info = s_zero;
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

template <typename T, int W, int RPT, int NT>
hipError_t launch_leaf(hipStream_t s, int G, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k,
                       int32_t* info, LeafSlots* ws, uint32_t epoch, int64_t oc_lo, int64_t oc_hi) {
  hipLaunchKernelGGL((k_panel_leaf<T, W, RPT, NT>), dim3(G), dim3(NT), 0, s, r, w, P, ld, ipiv, k, info, ws, epoch,
                     oc_lo, oc_hi);
  return hipGetLastError();
}

}  // namespace

hipError_t reset_flags(hipStream_t s, LeafSlots* ws) {
  hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(256), 0, s, ws);
  return hipGetLastError();
}

namespace {
constexpr int kLeafThreads = 256;
// rows per thread: fewest workgroups (cheapest exchange) that keep the block
// in registers
// rows per thread: four at every height (the leaf is one fully unrolled
// W = 16 instantiation per precision; narrower leaves are masked)
int leaf_rpt(int64_t) { return 4; }
}  // namespace

int panel_groups(int64_t r) {
  const int rpt = leaf_rpt(r);
  return (int)((r + (int64_t)kLeafThreads * rpt - 1) / ((int64_t)kLeafThreads * rpt));
}

template <typename T>
hipError_t panel_leaf(hipStream_t s, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k, int32_t* info,
                      LeafSlots* ws, uint32_t epoch, int64_t oc_lo, int64_t oc_hi) {
  if (w <= 0 || r <= 0) return hipSuccess;
  if (w > 16 || oc_lo > 0 || oc_hi < w) return hipErrorInvalidValue;
  constexpr int NT = kLeafThreads;
  const int rpt = leaf_rpt(r);
  const int64_t G64 = (r + (int64_t)NT * rpt - 1) / ((int64_t)NT * rpt);
  if (G64 > kLeafMaxGroups) return hipErrorInvalidValue;
  const int G = (int)G64;
  const int64_t n_other = -oc_lo + (oc_hi - w);
  if (n_other > (int64_t)kMaxOther * G * NT) return hipErrorInvalidValue;
  return launch_leaf<T, 16, 4, NT>(s, G, r, w, P, ld, ipiv, k, info, ws, epoch, oc_lo, oc_hi);
}

template hipError_t panel_leaf<double>(hipStream_t, int64_t, int, double*, int64_t, int32_t*, int64_t, int32_t*,
                                       LeafSlots*, uint32_t, int64_t, int64_t);
template hipError_t panel_leaf<float>(hipStream_t, int64_t, int, float*, int64_t, int32_t*, int64_t, int32_t*,
                                      LeafSlots*, uint32_t, int64_t, int64_t);

}  // namespace lupp
