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
//      (and, from the owner of row j, row j) as 64-bit device-coherent words
//      that each carry the column's tag -- no store fence, no separate flag.
//      One wavefront polls the G three-word headers (|a|, row) until all tags
//      are current, picks the winner, then reads the winner's row and row j
//      (tag-checked): two light round trips;
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
  static_assert(W <= kLeafMaxWidth, "leaf wider than the exchange records");
  constexpr int NW = NT / 64;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int64_t rbase = (int64_t)g * NT * RPT;

  // double-buffered by column parity: a buffer written for column j is read
  // only before the first barrier of column j + 1
  __shared__ T s_wrow[2][NW][W];  // each wavefront's candidate row
  __shared__ T s_rowj[2][W];      // row j before the interchange
  __shared__ T s_prow[2][W];      // the pivot row (G > 1)
  __shared__ double s_wv[2][NW];
  __shared__ uint32_t s_wi[2][NW];
  __shared__ uint32_t s_bi[2];
  __shared__ int s_broken;
  __shared__ int32_t s_ipiv[W];
  __shared__ int32_t s_zero;
  __shared__ uint32_t s_words[3 * kLeafMaxGroups];

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
      // 1. this thread's candidate: the first maximal |a| among its rows >= j
      //    (its rows increase with q), then the wavefront's, exactly: the
      //    largest |a|, then the lowest row holding it
      double lv = -1.0;
      uint32_t li = kNone;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        const double v = fabs((double)a[q][j]);
        if (i >= j && i < r && v > lv) {
          lv = v;
          li = (uint32_t)i;
        }
      }
      const double wm = wave_max_f64(lv);
      const uint32_t wi = wave_min_u32((lv == wm) ? li : kNone);
      // the wavefront's candidate row and row j go to LDS with the candidate
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t i = rbase + q * NT + tid;
        if (i == (int64_t)wi) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_wrow[par][wave][c] = a[q][c];
        }
        if (i == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_rowj[par][c] = a[q][c];
        }
      }
      if (lane == 0) {
        s_wv[par][wave] = wm;
        s_wi[par][wave] = wi;
      }
      lds_barrier();
      // 2. the workgroup's candidate (every thread, the same order)
      double bv = s_wv[par][0];
      uint32_t bi = s_wi[par][0];
      int bw = 0;
#pragma unroll
      for (int q = 1; q < NW; ++q) {
        const double v = s_wv[par][q];
        const uint32_t ii = s_wi[par][q];
        if (v > bv || (v == bv && ii < bi)) {
          bv = v;
          bi = ii;
          bw = q;
        }
      }
      const T* prow;
      uint32_t pu;
      if (G == 1) {
        prow = s_wrow[par][bw];
        pu = bi;
      } else {
        // one wavefront publishes this workgroup's tagged record (and, in
        // workgroup 0, row j), then reads every workgroup's record until all
        // tags are current: one round trip in the common case
        if (wave == 0) {
          const uint32_t tag = epoch + (uint32_t)j + 1u;
          const uint64_t th = (uint64_t)tag << 32;
          if (lane < kLeafRecWords) {
            uint32_t pay;
            if (lane < 2) {
              const uint64_t vb = (uint64_t)__double_as_longlong(bv);
              pay = lane == 0 ? (uint32_t)(vb >> 32) : (uint32_t)vb;
            } else if (lane == 2) {
              pay = bi;
            } else {
              const int e = lane - 3;
              const uint64_t db = (uint64_t)__double_as_longlong((double)s_wrow[par][bw][e >> 1]);
              pay = (e & 1) ? (uint32_t)db : (uint32_t)(db >> 32);
            }
            st_u64(&ws->rec[par][g][lane], th | pay);
          }
          if (g == 0 && lane < 2 * W) {
            const uint64_t db = (uint64_t)__double_as_longlong((double)s_rowj[par][lane >> 1]);
            st_u64(&ws->rowj[par][lane], th | ((lane & 1) ? (uint32_t)db : (uint32_t)(db >> 32)));
          }
          // (a) the G headers (|a| and row) until every tag is current
          const int nhead = 3 * G;
          if (!s_broken) {
            long spins = 0;
            for (;;) {
              bool ok = true;
              for (int e = lane; e < nhead; e += 64) {
                const uint64_t v = ld_u64(&ws->rec[par][e / 3][e % 3]);
                ok &= (uint32_t)(v >> 32) == tag;
                s_words[e] = (uint32_t)v;
              }
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
          double cv = -1.0;
          uint32_t ci = kNone;
          for (int q = lane; q < G; q += 64) {
            const uint32_t* wq = &s_words[3 * q];
            const double v = __longlong_as_double((long long)(((uint64_t)wq[0] << 32) | wq[1]));
            const uint32_t ii = wq[2];
            if (v > cv || (v == cv && ii < ci)) {
              cv = v;
              ci = ii;
            }
          }
          const double gm = wave_max_f64(cv);
          const uint32_t gi = wave_min_u32((cv == gm) ? ci : kNone);
          // the winning row identifies its workgroup
          const int gw = (gi == kNone) ? 0 : (int)((int64_t)gi / ((int64_t)NT * RPT));
          // (b) the winner's row and (outside workgroup 0) row j, tag-checked
          const bool need = lane < 2 * W || (g != 0 && lane < 4 * W);
          uint64_t rv = 0;
          if (!s_broken) {
            long spins = 0;
            for (;;) {
              bool ok = true;
              if (need) {
                rv = (lane < 2 * W) ? ld_u64(&ws->rec[par][gw][3 + lane]) : ld_u64(&ws->rowj[par][lane - 2 * W]);
                ok = (uint32_t)(rv >> 32) == tag;
              }
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
          // two 32-bit halves per value: even lane high, odd lane low
          const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)rv, 1, 64);
          if (need && (lane & 1) == 0) {
            const double d = __longlong_as_double((long long)(((uint64_t)(uint32_t)rv << 32) | lo));
            if (lane < 2 * W) s_prow[par][lane >> 1] = (T)d;
            else s_rowj[par][(lane - 2 * W) >> 1] = (T)d;
          }
          if (lane == 0) s_bi[par] = gi;
        }
        lds_barrier();
        prow = s_prow[par];
        pu = s_bi[par];
      }

      // 3. interchange, scale, update (a winner outside the block can only
      // come from NaN input: keep the diagonal row then)
      int64_t piv = (int64_t)pu;
      if (pu == kNone || piv < j || piv >= r) piv = j;
      const T pv = prow[j];
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
            for (int c = 0; c < W; ++c) a[q][c] = s_rowj[par][c];
          } else if (i == j) {
#pragma unroll
            for (int c = 0; c < W; ++c) a[q][c] = prow[c];
          }
          if (i > j && i < r) {
            const T l = a[q][j] / pv;
            a[q][j] = l;
#pragma unroll
            for (int c = 0; c < W; ++c)
              if (c > j) a[q][c] = a[q][c] - l * prow[c];
          }
        }
      }
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

// clears every tag (tag 0 is never issued), so records left from before an
// epoch wrap-around cannot match a new tag
__global__ void k_reset_flags(LeafSlots* ws) {
  for (int i = threadIdx.x; i < kLeafMaxGroups; i += blockDim.x) ws->flags[i] = 0;
  uint64_t* rec = &ws->rec[0][0][0];
  for (int i = threadIdx.x; i < 2 * kLeafMaxGroups * kLeafRecStride; i += blockDim.x) rec[i] = 0;
  for (int i = threadIdx.x; i < 4 * kLeafMaxWidth; i += blockDim.x) (&ws->rowj[0][0])[i] = 0;
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
