// Column-block ("panel") factorization with partial pivoting.  The paper
// singles this step out as the one that limits a blocked LU: it works on few
// data and every other step waits for it (Section 4.1).  Its latency is a
// chain of w dependent pivot decisions, each a reduction over all r rows.
//
// Design (gfx950): one cooperative launch factors a column block of up to 256
// columns.  G workgroups of 1024 threads split the r rows, one row per thread.
// The block is processed in chunks of 16 columns, left-looking:
//   0. a grid barrier (per-workgroup tags) makes the previous chunk's stores
//      visible everywhere;
//   1. every thread loads its row of the chunk into registers;
//   2. workgroup 0 forward-substitutes the chunk's rows above the diagonal
//      (U12 := inv(L11) A12, one row per step) and publishes them; every
//      workgroup then updates its rows below with the finished columns
//      (A22 -= L21 U12), streaming L21 with four loads in flight per thread;
//   3. the chunk is factored column by column with the rows in registers:
//      each wavefront reduces its candidates exactly (largest |a|, then the
//      lowest row, two DPP reductions); within a workgroup one barrier per
//      column; across workgroups each publishes a record of 64-bit
//      device-coherent words that carry the column's tag, and one wavefront
//      polls the G three-word headers (|a|, row) until every tag is current,
//      picks the winner, then reads the winner's row and row j (tag-checked);
//      interchange, true-division scaling and the rank-1 update of the
//      chunk follow in registers;
//   4. the chunk is written back.
// Each interchange is also applied to the other columns of the block and of
// the enclosing column block by threads that own one such column each; a
// step's loads are issued as soon as the pivot is known and its stores in
// the next step.  All accesses that another workgroup may read within the
// launch bypass the non-coherent caches (agent scope).  Waits are bounded: an
// expired wait sets ws->err and the kernel finishes.
#include "common.h"
#include "wave.h"

namespace lupp {
namespace {

constexpr long kSpinLimit = 1L << 22;
constexpr int kMaxOther = 1;  // other columns per thread (enclosing block <= 1024 columns <= threads)

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
__device__ __forceinline__ void st_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// element loads and stores that bypass the non-coherent caches
template <typename T>
__device__ __forceinline__ T ldc(const T* p);
template <>
__device__ __forceinline__ double ldc<double>(const double* p) { return ld_f64(p); }
template <>
__device__ __forceinline__ float ldc<float>(const float* p) { return __uint_as_float(ld_u32((const uint32_t*)p)); }
template <typename T>
__device__ __forceinline__ void stc(T* p, T v);
template <>
__device__ __forceinline__ void stc<double>(double* p, double v) { st_f64(p, v); }
template <>
__device__ __forceinline__ void stc<float>(float* p, float v) { st_u32((uint32_t*)p, __float_as_uint(v)); }

// wait until this thread's stores have completed at the coherence point
__device__ __forceinline__ void release_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}



template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_panel_block(int64_t r, int wt, T* __restrict__ P, int64_t ld,
                                                    int32_t* __restrict__ ipiv, int64_t k,
                                                    int32_t* __restrict__ info, LeafSlots* __restrict__ ws,
                                                    uint32_t epoch, int64_t oc_lo, int64_t oc_hi) {
  constexpr int W = 16;  // chunk width
  static_assert(W <= kLeafMaxWidth, "chunk wider than the exchange records");
  constexpr int NW = NT / 64;
  constexpr int PF = 4;  // L loads in flight per thread in the left-looking update
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int i = g * NT + tid;  // this thread's row (block-relative; r < 2^31)
  const bool rok = i < r;

  // double-buffered by column parity: a buffer written for column j is read
  // only before the first barrier of column j + 1
  __shared__ T s_wrow[2][NW][W];  // each wavefront's candidate row
  __shared__ T s_rowj[2][W];      // row j before the interchange
  __shared__ T s_prow[2][W];      // the pivot row (G > 1)
  __shared__ double s_wv[2][NW];
  __shared__ uint32_t s_wi[2][NW];
  __shared__ uint32_t s_bi[2];
  __shared__ int s_broken;
  __shared__ int32_t s_ipiv[kBlockMaxWidth];
  __shared__ int32_t s_zero;
  __shared__ T s_u[kBlockMaxWidth][W];  // the chunk's rows above the diagonal
  __shared__ T s_lp[2][W][kBlockMaxWidth];  // workgroup 0: 16-column panels of L11, double-buffered

  if (tid == 0) {
    s_broken = 0;
    s_zero = 0;
  }
  __syncthreads();

  // every workgroup waits until all workgroups have reached this point with
  // their stores completed
  auto grid_barrier = [&](uint32_t tag) {
    release_stores();
    __syncthreads();
    if (wave == 0) {
      if (lane == 0) st_u32(&ws->flags[g], tag);
      if (!s_broken) {
        long spins = 0;
        for (;;) {
          bool ok = true;
          for (int q = lane; q < G; q += 64) ok &= ld_u32(&ws->flags[q]) >= tag;
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
    __syncthreads();
  };

  const int nch = (wt + W - 1) / W;
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = ch * W;
    const int cw = (wt - c0 < W) ? (wt - c0) : W;
    const uint32_t tbase = epoch + 1u + (uint32_t)ch * (W + 2);
    // ---- 0. the previous chunk's stores are visible to every workgroup
    if (ch > 0) grid_barrier(tbase + W);
    // ---- 1. this thread's row of the chunk
    T a[W];
#pragma unroll
    for (int c = 0; c < W; ++c) a[c] = (rok && c < cw) ? ldc(P + i + (int64_t)(c0 + c) * ld) : T(0);

    // ---- 2. left-looking update with the finished columns 0 .. c0-1
    if (c0 > 0) {
      if (g == 0) {
        // rows 0 .. c0-1: U12 = inv(L11) A12 in 16-row blocks.  Panel b of
        // L11 (rows 16b .. c0-1, columns 16b .. 16b+15) is staged in LDS, the
        // next one's loads in flight meanwhile; 16 lanes solve the block's
        // rows column-wise (x_i -= l_ik x_k in increasing k), then every row
        // below subtracts the block's contribution in increasing k, so each
        // row sees its terms in the order of plain forward substitution.
        // The barriers wait for LDS traffic only, not for the loads in flight.
        constexpr int PL = (W * kBlockMaxWidth) / NT;  // panel elements per thread
        const int nbk = c0 / 16;
        T pl[PL];
        auto issue = [&](int b) {
#pragma unroll
          for (int q = 0; q < PL; ++q) {
            const int e = tid + q * NT;
            const int kk = e / kBlockMaxWidth, row = 16 * b + (e % kBlockMaxWidth);
            pl[q] = (row < c0) ? ldc(P + row + (int64_t)(16 * b + kk) * ld) : T(0);
          }
        };
        auto place = [&](int buf) {
#pragma unroll
          for (int q = 0; q < PL; ++q) {
            const int e = tid + q * NT;
            s_lp[buf][e / kBlockMaxWidth][e % kBlockMaxWidth] = pl[q];
          }
        };
        issue(0);
        if (tid < c0) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_u[tid][c] = a[c];
        }
        place(0);
        lds_barrier();
        for (int bb = 0; bb < nbk; ++bb) {
          const int buf = bb & 1, row0 = 16 * bb;
          if (bb + 1 < nbk) issue(bb + 1);
          if (tid < 16 * W) {
            // thread (ii, c) = (tid & 15, tid >> 4) holds row row0+ii of column
            // c; step kk broadcasts row kk inside the 16-lane row
            const int ii = tid & 15, c = tid >> 4;
            T x = s_u[row0 + ii][c];
            static_for<0, 16>([&](auto kc) {
              constexpr int kk = decltype(kc)::value;
              const T xk = row_bcast<kk>(x);
              const T nx = x - s_lp[buf][kk][ii] * xk;
              x = (ii > kk) ? nx : x;
            });
            s_u[row0 + ii][c] = x;
          }
          lds_barrier();
          if (tid >= row0 + 16 && tid < c0) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
              const T l = s_lp[buf][kk][tid - row0];
#pragma unroll
              for (int c = 0; c < W; ++c) a[c] = a[c] - l * s_u[row0 + kk][c];
              __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int c = 0; c < W; ++c) s_u[tid][c] = a[c];
          }
          if (bb + 1 < nbk) place(buf ^ 1);
          lds_barrier();
        }
        if (tid < c0) {
#pragma unroll
          for (int c = 0; c < W; ++c) a[c] = s_u[tid][c];
        }
        // publish U12 for the other workgroups
        if (tid < c0) {
#pragma unroll
          for (int c = 0; c < W; ++c)
            if (c < cw) stc(P + tid + (int64_t)(c0 + c) * ld, a[c]);
        }
        release_stores();
        __syncthreads();
        if (tid == 0) st_u32(&ws->uflag, tbase + W + 1);
      } else {
        if (wave == 0 && !s_broken) {
          long spins = 0;
          for (;;) {
            const bool ok = ld_u32(&ws->uflag) >= tbase + W + 1;
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
        __syncthreads();
        for (int e = tid; e < c0 * W; e += NT) {
          const int pr = e / W, c = e % W;
          s_u[pr][c] = (c < cw) ? ldc(P + pr + (int64_t)(c0 + c) * ld) : T(0);
        }
        __syncthreads();
      }
      // rows c0 .. r-1: A22 -= L21 U12
      if (rok && i >= c0) {
        T lr[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) lr[u] = (u < c0) ? ldc(P + i + (int64_t)u * ld) : T(0);
        for (int pb = 0; pb < c0; pb += PF) {
          T cur[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) cur[u] = lr[u];
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            const int p = pb + PF + u;
            lr[u] = (p < c0) ? ldc(P + i + (int64_t)p * ld) : T(0);
          }
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            const int p = pb + u;
            if (p < c0) {
#pragma unroll
              for (int c = 0; c < W; ++c) a[c] = a[c] - cur[u] * s_u[p][c];
            }
          }
        }
      }
    }

    // ---- 3. the chunk's columns, one pivot at a time
    // other columns of the enclosing block owned by this thread: [oc_lo, c0)
    // and [c0 + cw, oc_hi), relative to P
    const int64_t n_left = (int64_t)c0 - oc_lo, n_other = n_left + (oc_hi - c0 - cw);
    const int64_t gt = (int64_t)g * NT + tid, gstride = (int64_t)G * NT;
    T* ocol[kMaxOther];
    bool own[kMaxOther];
#pragma unroll
    for (int u = 0; u < kMaxOther; ++u) {
      const int64_t q = gt + u * gstride;
      own[u] = q < n_other;
      const int64_t c = (q < n_left) ? (oc_lo + q) : (c0 + cw + (q - n_left));
      ocol[u] = P + (own[u] ? c : 0) * ld;
    }
    bool pend = false;
    int prj = 0, prp = 0;
    T pvj[kMaxOther], pvp[kMaxOther];

#pragma clang loop unroll(full)
    for (int j = 0; j < W; ++j) {
      if (j < cw) {
        const int par = j & 1;
        const int jg = c0 + j;
        // 1. candidates: the largest |a| over rows >= jg, then the lowest row
        const double lv = (rok && i >= jg) ? fabs((double)a[j]) : -1.0;
        const uint32_t li = (rok && i >= jg) ? (uint32_t)i : kNone;
        const double wm = wave_max_f64(lv);
        // rows grow with the lane: the lowest lane holding the maximum has the lowest row
        const uint64_t hit = __ballot(li != kNone && lv == wm);
        const uint32_t wi = hit ? (uint32_t)__builtin_amdgcn_readlane((int)li, (int)__builtin_ctzll(hit)) : kNone;
        if ((uint32_t)i == wi) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_wrow[par][wave][c] = a[c];
        }
        if (i == jg) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_rowj[par][c] = a[c];
        }
        if (lane == 0) {
          s_wv[par][wave] = wm;
          s_wi[par][wave] = wi;
        }
        lds_barrier();
        // 2. the workgroup's candidate (every thread, the same order): each
        // 16-lane row of a wavefront reads the NW wavefront candidates and
        // reduces them with four DPP steps
        double bv;
        uint32_t bi;
        int bw;
        {
          static_assert(NW <= 16, "one wavefront candidate per lane of a 16-lane row");
          const int q = lane & 15;
          uint32_t khi = 0, klo = 0, kidx = kNone;
          if (q < NW) {
            const double v = s_wv[par][q];
            const uint32_t ii = s_wi[par][q];
            if (ii != kNone && v >= 0.0) {
              const uint64_t vb = (uint64_t)__double_as_longlong(v);
              khi = (uint32_t)(vb >> 32);
              klo = (uint32_t)vb;
              kidx = ii;
            }
          }
          dpp_step<0xB1>(khi, klo, kidx);
          dpp_step<0x4E>(khi, klo, kidx);
          dpp_step<0x141>(khi, klo, kidx);
          dpp_step<0x140>(khi, klo, kidx);
          bi = kidx;
          bv = (kidx == kNone) ? -1.0 : __longlong_as_double((long long)(((uint64_t)khi << 32) | klo));
          bw = (kidx == kNone) ? 0 : (int)((kidx - (uint32_t)g * NT) / 64u);
        }
        const T* prow;
        uint32_t pu;
        if (G == 1) {
          prow = s_wrow[par][bw];
          pu = bi;
        } else {
          if (wave == 0) {
            const uint32_t tag = tbase + (uint32_t)j;
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
            // (a) the G headers until every tag is current: lane q holds the
            // three header words of workgroup q (and then of q + 64), loaded
            // together, and keeps the better candidate
            uint32_t khi = 0, klo = 0, kidx = kNone;
            if (!s_broken) {
              long spins = 0;
              for (;;) {
                bool ok = true;
                khi = 0;
                klo = 0;
                kidx = kNone;
                for (int q = lane; q < G; q += 64) {
                  const uint64_t h0 = ld_u64(&ws->rec[par][q][0]);
                  const uint64_t h1 = ld_u64(&ws->rec[par][q][1]);
                  const uint64_t h2 = ld_u64(&ws->rec[par][q][2]);
                  ok &= (uint32_t)(h0 >> 32) == tag && (uint32_t)(h1 >> 32) == tag && (uint32_t)(h2 >> 32) == tag;
                  const uint32_t chi = (uint32_t)h0, clo = (uint32_t)h1, cidx = (uint32_t)h2;
                  const double v = __longlong_as_double((long long)(((uint64_t)chi << 32) | clo));
                  if (cidx != kNone && v >= 0.0 && key_better(chi, clo, cidx, khi, klo, kidx)) {
                    khi = chi;
                    klo = clo;
                    kidx = cidx;
                  }
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
            double gv = kidx == kNone ? -1.0 : __longlong_as_double((long long)(((uint64_t)khi << 32) | klo));
            int64_t gi64 = kidx == kNone ? INT64_MAX : (int64_t)kidx;
            wave_argmax(gv, gi64);
            const uint32_t gi = (gi64 == INT64_MAX) ? kNone : (uint32_t)gi64;
            const int gw = (gi == kNone) ? 0 : (int)((int64_t)gi / NT);
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
        int piv = (int)pu;
        if (pu == kNone || piv < jg || (int64_t)piv >= r) piv = jg;
        const T pv = prow[j];
        if (tid == 0) {
          s_ipiv[jg] = (int32_t)(k + piv + 1);
          if (pv == T(0) && s_zero == 0) s_zero = (int32_t)(k + jg + 1);
        }
        // the same interchange on the other columns: stores of the previous
        // step, loads of this one
        if (pend) {
#pragma unroll
          for (int u = 0; u < kMaxOther; ++u)
            if (own[u]) {
              stc(ocol[u] + prj, pvp[u]);
              stc(ocol[u] + prp, pvj[u]);
            }
          pend = false;
        }
        if (piv != jg && pv != T(0)) {
#pragma unroll
          for (int u = 0; u < kMaxOther; ++u)
            if (own[u]) {
              pvj[u] = ldc(ocol[u] + jg);
              pvp[u] = ldc(ocol[u] + piv);
            }
          pend = true;
          prj = jg;
          prp = piv;
        }
        if (pv != T(0)) {
          if (i == piv && piv != jg) {
#pragma unroll
            for (int c = 0; c < W; ++c) a[c] = s_rowj[par][c];
          } else if (i == jg) {
#pragma unroll
            for (int c = 0; c < W; ++c) a[c] = prow[c];
          }
          if (rok && i > jg) {
            if constexpr (sizeof(T) == 4) {
              // the pivot row's values read before the division, so the reads
              // are in flight during it (FP32 only: in FP64 the values do
              // not fit the registers beside the row)
              T pr[W];
#pragma unroll
              for (int c = 0; c < W; ++c) pr[c] = (c > j) ? prow[c] : T(0);
              const T l = a[j] / pv;
              a[j] = l;
#pragma unroll
              for (int c = 0; c < W; ++c)
                if (c > j) a[c] = a[c] - l * pr[c];
            } else {
              const T l = a[j] / pv;
              a[j] = l;
#pragma unroll
              for (int c = 0; c < W; ++c)
                if (c > j) a[c] = a[c] - l * prow[c];
            }
          }
        }
      }
    }
    if (pend) {
#pragma unroll
      for (int u = 0; u < kMaxOther; ++u)
        if (own[u]) {
          stc(ocol[u] + prj, pvp[u]);
          stc(ocol[u] + prp, pvj[u]);
        }
    }
    // ---- 4. the chunk back (every row)
    if (rok) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < cw) stc(P + i + (int64_t)(c0 + c) * ld, a[c]);
    }
  }

  lds_barrier();  // s_ipiv / s_zero complete
  if (g == 0) {
    for (int jj = tid; jj < wt; jj += NT) ipiv[k + jj] = s_ipiv[jj];
    if (tid == 0 && s_zero != 0 && *info == 0) *info = s_zero;
  }
}

// clears every tag (tag 0 is never issued), so records left from before an
// epoch wrap-around cannot match a new tag
__global__ void k_reset_flags(LeafSlots* ws) {
  for (int i = threadIdx.x; i < kLeafMaxGroups; i += blockDim.x) ws->flags[i] = 0;
  if (threadIdx.x == 0) ws->uflag = 0;
  uint64_t* rec = &ws->rec[0][0][0];
  for (int i = threadIdx.x; i < 2 * kLeafMaxGroups * kLeafRecStride; i += blockDim.x) rec[i] = 0;
  for (int i = threadIdx.x; i < 4 * kLeafMaxWidth; i += blockDim.x) (&ws->rowj[0][0])[i] = 0;
}

constexpr int kBlockThreads = 1024;

}  // namespace

hipError_t reset_flags(hipStream_t s, LeafSlots* ws) {
  hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(256), 0, s, ws);
  return hipGetLastError();
}

int panel_groups(int64_t r) { return (int)((r + kBlockThreads - 1) / kBlockThreads); }

uint32_t block_tags(int w) { return (uint32_t)(((w + 15) / 16) * 18 + 2); }

template <typename T>
hipError_t panel_block(hipStream_t s, int64_t r, int w, T* P, int64_t ld, int32_t* ipiv, int64_t k, int32_t* info,
                       LeafSlots* ws, uint32_t epoch, int64_t oc_lo, int64_t oc_hi) {
  if (w <= 0 || r <= 0) return hipSuccess;
  if (w > kBlockMaxWidth || r < w || oc_lo > 0 || oc_hi < w) return hipErrorInvalidValue;
  const int64_t G64 = (r + kBlockThreads - 1) / kBlockThreads;
  if (G64 > kLeafMaxGroups) return hipErrorInvalidValue;
  const int G = (int)G64;
  if (oc_hi - oc_lo > (int64_t)kMaxOther * G * kBlockThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_panel_block<T, kBlockThreads>), dim3(G), dim3(kBlockThreads), 0, s, r, w, P, ld, ipiv, k,
                     info, ws, epoch, oc_lo, oc_hi);
  return hipGetLastError();
}

template hipError_t panel_block<double>(hipStream_t, int64_t, int, double*, int64_t, int32_t*, int64_t, int32_t*,
                                        LeafSlots*, uint32_t, int64_t, int64_t);
template hipError_t panel_block<float>(hipStream_t, int64_t, int, float*, int64_t, int32_t*, int64_t, int32_t*,
                                       LeafSlots*, uint32_t, int64_t, int64_t);

}  // namespace lupp
