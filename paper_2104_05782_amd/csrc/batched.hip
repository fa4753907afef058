// Batched LU with partial pivoting and solve for many small systems
// (order n <= 128), one workgroup per system with the system held in
// registers.
//
// Each system is factored with LAPACK's conventions for partial pivoting
// (the column step of Section 4.1, one column at a time, at the scale of one
// workgroup) applied to the augmented matrix [A | b], so that the row
// interchanges and the elimination also carry b to L^{-1} P b; a backward
// substitution with U then gives x (skipped, as in LAPACK's gesv, when a
// pivot is exactly zero).
//
// Scheduling: a binning kernel sorts the systems into size classes (up to
// six, by upper bounds on n), each served by one persistent launch of a
// kernel shape (wavefronts per system, row slots per lane, columns per
// wavefront) whose workgroups take the class's systems in round robin (no
// shared counter: thousands of workgroups contending for one global atomic
// cost more than the small systems themselves).  A CU's register file
// (512 KB) holds several systems of every class, where its LDS (160 KB) would
// hold one of the largest.  The classes are launched on their own streams so
// that the short classes fill the CUs the long ones leave idle (measured: one
// launch of the largest shape for the whole batch takes 1.5x the time of the
// per-class launches).  The class bounds, the shape of each class and its grid
// form the handle's schedule, which the package's autotuner chooses by timing
// graph replays of this call; the default is four classes (n <= 32, 64, 96,
// 128).  No host synchronization or allocation happens per call
// (graph-capturable once the workspace exists for the batch size).
#include <mutex>
#include <utility>

#include "handle.h"
#include "wave.h"

namespace lupp {

constexpr int kMaxClasses = 6;
constexpr int kBatchMaxN = 128;
// Bound on a wavefront's wait for a published step (iterations of a ~64-cycle
// sleep, about 0.1 s): a wait that long means a fault in the schedule, and the
// system is then abandoned with info = kStalled instead of hanging the GPU.
constexpr int kSpinLimit = 1 << 22;
constexpr int kStalled = -1000;

// Kernel shapes: NW wavefronts per system, R row slots per lane (rows l and
// l + 64), C columns per wavefront; a shape holds orders up to
// min(64 R, NW C - 1) (b is one more column).
struct Shape {
  int nw, r, c;
};
constexpr Shape kShapes[] = {{1, 1, 17}, {1, 1, 33}, {2, 1, 33}, {1, 1, 65}, {4, 1, 17},
                             {4, 2, 25}, {2, 2, 49}, {8, 2, 13}, {4, 2, 33}, {8, 2, 17}};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
constexpr int shape_nmax(int v) {
  return 64 * kShapes[v].r < kShapes[v].nw * kShapes[v].c - 1 ? 64 * kShapes[v].r : kShapes[v].nw * kShapes[v].c - 1;
}

// Schedule of one precision: class c holds the orders in (ub[c-1], ub[c]].
struct Schedule {
  int nclass = 0;
  int ub[kMaxClasses] = {};
  int shape[kMaxClasses] = {};
  int grid_pct[kMaxClasses] = {};
};

// Workspace of the batched path: per-class system lists and counters.
struct BatchWs {
  int64_t capacity = 0;
  int32_t* list = nullptr;  // capacity entries: system ids grouped by class
  int32_t* meta = nullptr;  // [0, kMaxClasses) counts, [kMaxClasses, 2 kMaxClasses) offsets
  hipStream_t streams[kMaxClasses] = {};
  hipEvent_t fork = nullptr, join[kMaxClasses] = {};
  int occ[2][kNumShapes] = {};  // resident workgroups per device, per (precision, shape)
  Schedule sched[2];            // FP64, FP32
};

// Class bounds as a kernel argument.
struct ClassBounds {
  int nclass;
  int ub[kMaxClasses];
};

namespace {

__device__ __forceinline__ int size_class(int n, const ClassBounds& cb) {
  int c = 0;
#pragma unroll
  for (int q = 0; q < kMaxClasses - 1; ++q)
    if (q < cb.nclass - 1 && n > cb.ub[q]) c = q + 1;
  return c;
}

// Sort systems into size classes.  One workgroup; the
// counters are updated once per wavefront and class (ballot + popcount), not
// once per system.
__global__ __launch_bounds__(1024) void k_batch_bin(int32_t batch, const int32_t* __restrict__ dn,
                                                    int32_t* __restrict__ list, int32_t* __restrict__ meta,
                                                    int32_t* __restrict__ info, ClassBounds cb) {
  __shared__ int cnt[kMaxClasses], cur[kMaxClasses], off[kMaxClasses];
  const int tid = threadIdx.x, lane = tid & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (tid < kMaxClasses) cnt[tid] = 0;
  __syncthreads();
  for (int base = 0; base < batch; base += 1024) {
    const int i = base + tid;
    int c = -1;
    if (i < batch) {
      const int n = dn[i];
      if (n >= 1 && n <= kBatchMaxN) c = size_class(n, cb);
      else info[i] = (n == 0) ? 0 : -1;  // empty system: nothing to do; bad order: rejected
    }
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
      const uint64_t b = __ballot(c == q);
      if (lane == 0 && b) atomicAdd(&cnt[q], __popcll(b));
    }
  }
  __syncthreads();
  if (tid == 0) {
    int o = 0;
    for (int c = 0; c < kMaxClasses; ++c) {
      off[c] = o;
      cur[c] = 0;
      meta[c] = cnt[c];
      meta[kMaxClasses + c] = o;
      o += cnt[c];
    }
  }
  __syncthreads();
  for (int base = 0; base < batch; base += 1024) {
    const int i = base + tid;
    int c = -1;
    if (i < batch) {
      const int n = dn[i];
      if (n >= 1 && n <= kBatchMaxN) c = size_class(n, cb);
    }
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
      const uint64_t b = __ballot(c == q);
      if (!b) continue;
      int at = 0;
      if (lane == 0) at = atomicAdd(&cur[q], __popcll(b));
      at = __builtin_amdgcn_readlane(at, 0);
      if (c == q) list[off[q] + at + __popcll(b & below)] = i;
    }
  }
}

// Pivot search on one column held as R row slots per lane (slot h*64 + lane):
// the largest |a| over the rows whose logical position is >= kp, the lowest
// logical row on ties (LAPACK's first maximum).  Returns the winner's slot
// and logical row; unless the pivot is zero, the column's candidate rows are
// replaced by their multipliers (true division, so |l| <= 1 exactly), which
// are also returned in lo (0 in every other slot).
template <int R, typename T>
__device__ __forceinline__ void pivot_column(T (&col)[R], T (&lo)[R], const int (&pos)[R], const bool (&valid)[R],
                                             int kp, int n, int lane, int& ps_out, int& p_out, bool& nz_out) {
  double a[R];
  double am = -1.0;
#pragma unroll
  for (int h = 0; h < R; ++h) {
    const bool cand = valid[h] && pos[h] >= kp;
    a[h] = cand ? (double)fabs(col[h]) : -1.0;
    am = fmax(am, a[h]);
  }
  const double m = wave_max_f64(am);
  uint32_t key = 0x7fffffffu;
#pragma unroll
  for (int h = 0; h < R; ++h)
    if (a[h] >= 0.0 && a[h] == m) key = min(key, (uint32_t)pos[h]);
  const uint32_t pm = wave_min_u32(key);
  const int p = (pm >= (uint32_t)kp && pm < (uint32_t)n) ? (int)pm : kp;  // kp only with NaN entries
  int ps = 0;
#pragma unroll
  for (int h = 0; h < R; ++h) {
    const uint64_t b = __ballot(valid[h] && pos[h] == p);
    if (b) ps = h * 64 + (int)__builtin_ctzll(b);
  }
  const T pv = (R == 1 || ps < 64) ? readlane_d(col[0], ps & 63) : readlane_d(col[R - 1], ps & 63);
  const bool nz = pv != T(0);
#pragma unroll
  for (int h = 0; h < R; ++h) {
    const bool cand = nz && valid[h] && pos[h] >= kp && h * 64 + lane != ps;
    const T q = col[h] / pv;
    lo[h] = cand ? q : T(0);
    if (cand) col[h] = q;
  }
  ps_out = ps;
  p_out = p;
  nz_out = nz;
}

// wavefronts per SIMD to ask of the register allocator: the matrix takes
// 2*R*C VGPRs in FP64, and what is left must hold the step's working set
template <int R, int C>
constexpr int kMinWaves = R * C > 80 ? 2 : (R * C > 40 ? 3 : 4);

// One system per workgroup of NW wavefronts, the whole augmented matrix
// [A | b] in registers: lane l holds rows l and (R = 2) l + 64, wavefront w
// holds columns w, w + NW, w + 2 NW, ... (C of them at most; b is column n).
//
// The factorization is LAPACK's unblocked right-looking elimination with
// partial pivoting (the column step of Section 4.1 applied one column at a
// time): for each column k, pivot search, interchange, scaling by the pivot
// and the rank-1 update of the columns to the right.  Rows never move: pos
// holds the logical row of each slot, an interchange exchanges two logical
// positions, and each row is written to its final position at the end.
//
// Step k:
//  - the multipliers and the pivot slot come from the wavefront owning
//    column k through LDS, published with a step counter: a wavefront waits
//    only for the step it needs, not for the other wavefronts' updates;
//  - each wavefront reads the pivot row's entries of its columns from the
//    pivot lane into scalar registers (v_readlane: 8 bytes per column, where
//    a broadcast through LDS would move 512 and saturate the LDS pipe) and
//    applies the rank-1 update as a chain of FMAs, register subscripts
//    static and no per-column branch (in a finished column it changes only
//    L entries, whose values were stored when the column was factored);
//  - lookahead: the owner of column k+1 applies step k to a copy of that
//    column first and publishes its pivot and multipliers before its chain,
//    so the pivot search overlaps the other wavefronts' updates.  The
//    multipliers are stored to the global matrix at the rows' slots (the
//    registers keep the column's updated values, the same as the copy's);
//    the final store takes L from there and U from the registers.
//
// The solve x = inv(U) c, c = L^{-1} P b being column n after the
// elimination, is a backward substitution by the wavefront holding b, with
// U read back from the stored factors (ten columns in flight) and the
// reciprocals of U's diagonal (skipped on a zero pivot, as in LAPACK's gesv).
//
// The multipliers on rows that are not below the pivot are zero: with finite
// values the FMA leaves such rows exactly unchanged (up to the sign of a
// zero); with +-Inf or NaN in the pivot row they become NaN where LAPACK
// would leave them.
template <typename T, int NW, int R, int C>
__global__ __launch_bounds__(64 * NW, (kMinWaves<R, C>)) void k_batch_lu(int cls, const int32_t* __restrict__ dn,
                                                      const int64_t* __restrict__ aoff, T* __restrict__ gA,
                                                      const int64_t* __restrict__ poff, int32_t* __restrict__ gpiv,
                                                      const int64_t* __restrict__ boff, T* __restrict__ gB,
                                                      int32_t* __restrict__ ginfo, const int32_t* __restrict__ list,
                                                      const int32_t* __restrict__ meta) {
  constexpr int NT = 64 * NW;
  // Published steps, a ring of kRing slots: slot k % kRing is rewritten for
  // step k + kRing, published by its owner only after every wavefront has
  // published a later step than k (each owns one of any NW consecutive
  // steps), hence has read slot k; kRing >= NW + 1 suffices.
  constexpr int kRing = NW < 8 ? 8 : 16;
  static_assert(kRing >= NW + 1, "ring of published steps too short");
  __shared__ T s_l[kRing][64 * R];  // multipliers
  __shared__ int s_pp[kRing][4];    // pivot slot, pivot's logical row, pivot nonzero
  __shared__ int s_done;            // steps published so far
  __shared__ int s_slot[kBatchMaxN], s_piv[kBatchMaxN];
  __shared__ int s_info;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
  const int count = meta[cls], first = meta[kMaxClasses + cls];

  // systems of the class in round robin over the persistent workgroups
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int sys = list[first + q];
    const int n = dn[sys];
    T* A = gA + aoff[sys];
    T* Bv = gB ? gB + boff[sys] : nullptr;
    if (tid == 0) {
      s_info = 0;
      s_done = 0;
    }
    __syncthreads();  // no wavefront sees the previous system's counter

    int pos[R];
    bool valid[R];
#pragma unroll
    for (int h = 0; h < R; ++h) {
      pos[h] = h * 64 + lane;
      valid[h] = pos[h] < n;
    }
    // ---- the system into registers (all loads issued before any use)
    T v[R][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = c * NW + w;
      const T* colp = j < n ? A + j * n : Bv;  // uniform column base
      const bool live = j < n || (j == n && Bv);
#pragma unroll
      for (int h = 0; h < R; ++h) {
        v[h][c] = T(0);
        if (live && valid[h]) v[h][c] = colp[(uint32_t)pos[h]];
      }
    }

    // ---- elimination
    T lm[R];
    int ps = 0, pp = 0;
    bool nz = true;
    // owner of column kp: record the pivot, store the multipliers at the
    // rows' slots, publish them to the other wavefronts
    auto publish = [&](int kp, const T(&col)[R], const T(&lo)[R], int ps1, int p1, bool nz1)
                       __attribute__((always_inline)) {
      if constexpr (NW > 1) {  // the step record first: the other wavefronts wait for it
        const int b = kp % kRing;
#pragma unroll
        for (int h = 0; h < R; ++h) s_l[b][h * 64 + lane] = lo[h];
        if (lane == 0) {
          s_pp[b][0] = ps1;
          s_pp[b][1] = p1;
          s_pp[b][2] = nz1 ? 1 : 0;
          __hip_atomic_store(&s_done, kp + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      if (lane == 0) {
        s_piv[kp] = p1;
        s_slot[kp] = ps1;
        if (!nz1 && s_info == 0) s_info = kp + 1;
      }
      T* colp = A + kp * n;
#pragma unroll
      for (int h = 0; h < R; ++h)
        if (valid[h] && pos[h] >= kp && h * 64 + lane != ps1) colp[h * 64 + lane] = col[h];
    };
    {
      T lo[R];
      int ps0 = 0, p0 = 0;
      bool nz0 = true;
      if (w == 0) {  // column 0: wavefront 0, local column 0
        T col[R];
#pragma unroll
        for (int h = 0; h < R; ++h) col[h] = v[h][0];
        pivot_column<R>(col, lo, pos, valid, 0, n, lane, ps0, p0, nz0);
        publish(0, col, lo, ps0, p0, nz0);
      }
      if constexpr (NW == 1) {
#pragma unroll
        for (int h = 0; h < R; ++h) lm[h] = lo[h];
        ps = ps0;
        pp = p0;
        nz = nz0;
      }
    }
    bool stalled = false;
    for (int k = 0; k < n; ++k) {
      if constexpr (NW > 1) {
        // wait for step k (bounded: on a stall the system is abandoned, so
        // that no wavefront can spin forever)
        int spins = 0;
        while (__builtin_amdgcn_readfirstlane(
                   __hip_atomic_load(&s_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) <= k) {
          if (++spins > kSpinLimit) {
            stalled = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (stalled) break;
        const int b = k % kRing;
        ps = __builtin_amdgcn_readfirstlane(s_pp[b][0]);
        pp = __builtin_amdgcn_readfirstlane(s_pp[b][1]);
        nz = __builtin_amdgcn_readfirstlane(s_pp[b][2]) != 0;
#pragma unroll
        for (int h = 0; h < R; ++h) lm[h] = s_l[b][h * 64 + lane];
      }
      // the interchange of step k: the pivot slot takes logical row k, the
      // slot that held row k takes the pivot's former position
      T ln[R];
#pragma unroll
      for (int h = 0; h < R; ++h) {
        const int sl = h * 64 + lane;
        pos[h] = (sl == ps) ? k : ((pos[h] == k) ? pp : pos[h]);
        ln[h] = (nz && valid[h] && pos[h] > k) ? -lm[h] : T(0);
      }
      const int hp = ps >> 6, lp = ps & 63;
      // lookahead on column k+1
      const int k1 = k + 1;
      const bool own1 = k1 < n && (NW == 1 || k1 % NW == w);
      T lo1[R];
      int ps1 = 0, p1 = 0;
      bool nz1 = true;
      if (own1) {
        // the lookahead is the critical path: its wavefront first in issue
        if constexpr (NW > 1) __builtin_amdgcn_s_setprio(3);
        const int c1 = k1 / NW;
        T col[R];
        dispatch<0, C>(c1, [&](auto ci) __attribute__((always_inline)) {
          constexpr int c = decltype(ci)::value;
#pragma unroll
          for (int h = 0; h < R; ++h) col[h] = v[h][c];
        });
        T u1 = readlane_d(col[0], lp);
        if constexpr (R > 1) {
          const T u1h = readlane_d(col[R - 1], lp);
          if (hp != 0) u1 = u1h;
        }
#pragma unroll
        for (int h = 0; h < R; ++h) col[h] = fma(ln[h], u1, col[h]);
        pivot_column<R>(col, lo1, pos, valid, k1, n, lane, ps1, p1, nz1);
        publish(k1, col, lo1, ps1, p1, nz1);
        if constexpr (NW > 1) __builtin_amdgcn_s_setprio(0);
      }
      // rank-1 update of the local columns from cmin on (the first column
      // right of k), in chunks of eight: the chunk's pivot-row entries are
      // read from the pivot lane into scalar registers (a branch on the
      // pivot's half that writes scalars only), then every lane applies its
      // FMAs.  A column left of cmin inside a live chunk is updated too: on
      // rows below the pivot it holds L entries, whose values were stored
      // when the column was factored, and the other rows have a zero
      // multiplier.
      const int cmin = k < w ? 0 : (k - w) / NW + 1;
      constexpr int CH = 8;
#pragma unroll
      for (int c0 = 0; c0 < C; c0 += CH) {
        if (c0 + CH - 1 >= cmin) {
          T u[CH];
          if (R == 1 || hp == 0) {
#pragma unroll
            for (int c = c0; c < c0 + CH && c < C; ++c) u[c - c0] = readlane_d(v[0][c], lp);
          } else {
#pragma unroll
            for (int c = c0; c < c0 + CH && c < C; ++c) u[c - c0] = readlane_d(v[R - 1][c], lp);
          }
#pragma unroll
          for (int c = c0; c < c0 + CH && c < C; ++c)
#pragma unroll
            for (int h = 0; h < R; ++h) v[h][c] = fma(ln[h], u[c - c0], v[h][c]);
        }
      }
      if constexpr (NW == 1) {
#pragma unroll
        for (int h = 0; h < R; ++h) lm[h] = lo1[h];
        ps = ps1;
        pp = p1;
        nz = nz1;
      }
    }
    if (stalled && lane == 0) s_info = kStalled;
    __syncthreads();
    const int info = s_info;
    if (info == kStalled) {  // nothing stored; info reports it
      if (tid == 0) ginfo[sys] = info;
      __syncthreads();
      continue;
    }

    // ---- L\U to its final rows: L (rows below the diagonal) from the
    // slot-ordered copy, U from the registers; every load of the workgroup
    // completes before any store moves a row
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = c * NW + w;
      if (j < n) {
        const T* colp = A + j * n;
#pragma unroll
        for (int h = 0; h < R; ++h)
          if (valid[h] && pos[h] > j) v[h][c] = colp[h * 64 + lane];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = c * NW + w;
      if (j < n) {
        T* colp = A + j * n;
#pragma unroll
        for (int h = 0; h < R; ++h)
          if (valid[h]) colp[(uint32_t)pos[h]] = v[h][c];
      }
    }

    // ---- x = inv(U) c by the wavefront holding b
    if (Bv && info == 0) {
      __syncthreads();  // the stored factors are visible to the workgroup
      if (w == n % NW) {
        T cv[R], rd[R];
        int sl[R];
        dispatch<0, C>(n / NW, [&](auto ci) __attribute__((always_inline)) {
          constexpr int c = decltype(ci)::value;
#pragma unroll
          for (int h = 0; h < R; ++h) cv[h] = v[h][c];
        });
#pragma unroll
        for (int h = 0; h < R; ++h) {
          rd[h] = valid[h] ? T(1) / A[pos[h] + pos[h] * n] : T(0);
          sl[h] = valid[h] ? s_slot[h * 64 + lane] : 0;
        }
        // U's column k at this lane's rows, D columns ahead; the loads are
        // unconditional (row and column clamped into the matrix) so that
        // none waits for the others, and the entries not above the diagonal
        // are masked where they are used
        constexpr int D = 10;
        int prow[R];
#pragma unroll
        for (int h = 0; h < R; ++h) prow[h] = valid[h] ? pos[h] : 0;
        T ub[D][R];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int kk = max(n - 1 - d, 0);
#pragma unroll
          for (int h = 0; h < R; ++h) ub[d][h] = A[prow[h] + kk * n];
        }
        for (int kb = n - 1; kb >= 0; kb -= D) {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const int k = kb - d;
            if (k < 0) break;
            const int sk = (R == 1 || k < 64) ? __builtin_amdgcn_readlane(sl[0], k & 63)
                                              : __builtin_amdgcn_readlane(sl[R - 1], k & 63);
            const int lk = sk & 63;
            const T xk = (R == 1 || sk < 64) ? readlane_d(cv[0], lk) * readlane_d(rd[0], lk)
                                             : readlane_d(cv[R - 1], lk) * readlane_d(rd[R - 1], lk);
#pragma unroll
            for (int h = 0; h < R; ++h) {
              const T t = fma(-ub[d][h], xk, cv[h]);
              cv[h] = (h * 64 + lane == sk) ? xk : ((valid[h] && pos[h] < k) ? t : cv[h]);
            }
            const int kn = max(k - D, 0);
#pragma unroll
            for (int h = 0; h < R; ++h) ub[d][h] = A[prow[h] + kn * n];
          }
        }
#pragma unroll
        for (int h = 0; h < R; ++h)
          if (valid[h]) Bv[pos[h]] = cv[h];
      }
    }
    int32_t* P = gpiv + poff[sys];
    for (int k = tid; k < n; k += NT) P[k] = s_piv[k] + 1;
    if (tid == 0) ginfo[sys] = info;
    __syncthreads();  // LDS reused by the next system
  }
}

template <typename T, int V>
constexpr const void* shape_kernel_of() {
  return (const void*)k_batch_lu<T, kShapes[V].nw, kShapes[V].r, kShapes[V].c>;
}
template <typename T, int... V>
const void* shape_kernel_at(int v, std::integer_sequence<int, V...>) {
  const void* table[] = {shape_kernel_of<T, V>()...};
  return table[v];
}
template <typename T>
const void* shape_kernel(int v) {
  return shape_kernel_at<T>(v, std::make_integer_sequence<int, kNumShapes>());
}
inline int shape_threads(int v) { return 64 * kShapes[v].nw; }

// The default schedule (four classes; measured by hand before the sweep
// existed): FP64 1x33, 2x33, 4x(2x25), 4x(2x33); FP32 the same with one
// wavefront of 65 columns for n <= 64.
Schedule default_schedule(int prec) {
  Schedule d;
  d.nclass = 4;
  const int ub[4] = {32, 64, 96, 128};
  const int sh[2][4] = {{1, 2, 5, 8}, {1, 3, 5, 8}};
  for (int c = 0; c < 4; ++c) {
    d.ub[c] = ub[c];
    d.shape[c] = sh[prec][c];
    d.grid_pct[c] = 100;
  }
  return d;
}

bool schedule_valid(const Schedule& s) {
  if (s.nclass < 1 || s.nclass > kMaxClasses) return false;
  int prev = 0;
  for (int c = 0; c < s.nclass; ++c) {
    if (s.ub[c] <= prev || s.ub[c] > kBatchMaxN) return false;
    if (s.shape[c] < 0 || s.shape[c] >= kNumShapes || shape_nmax(s.shape[c]) < s.ub[c]) return false;
    if (s.grid_pct[c] < 1 || s.grid_pct[c] > 100) return false;
    prev = s.ub[c];
  }
  return s.ub[s.nclass - 1] == kBatchMaxN;
}

template <typename T>
hipError_t setup_shape_occupancy(lupp_handle_t h, BatchWs* w, int prec) {
  int ncu = 0;
  LUPP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
  for (int v = 0; v < kNumShapes; ++v) {
    int occ = 0;
    LUPP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, shape_kernel<T>(v), shape_threads(v), 0));
    if (occ < 1) return hipErrorInvalidConfiguration;
    w->occ[prec][v] = occ * ncu;
  }
  return hipSuccess;
}

}  // namespace

void free_batched(lupp_handle_t h) {
  BatchWs* w = h->batch;
  if (!w) return;
  for (int c = 0; c < kMaxClasses; ++c) {
    if (w->streams[c]) (void)hipStreamSynchronize(w->streams[c]);
    if (w->join[c]) (void)hipEventDestroy(w->join[c]);
    if (w->streams[c]) (void)hipStreamDestroy(w->streams[c]);
  }
  if (w->fork) (void)hipEventDestroy(w->fork);
  if (w->list) (void)hipFree(w->list);
  delete w;
  h->batch = nullptr;
}

size_t batch_workspace_bytes(int64_t batch) { return (size_t)(batch < 1024 ? 1024 : batch) * 4 + 256; }

namespace {

// Scratch of the allocation-free entry point: the class list (one int per
// system) followed by the eight class counters and offsets, for at most
// kNoAllocMaxBatch systems.  Each device holds one copy until the process
// ends; every call on that device shares it.  Host code never passes the
// array's name to a kernel: it uses the device address looked up once per
// device at handle creation (g_scratch).
constexpr int64_t kNoAllocMaxBatch = 1 << 20;
constexpr int kScratchMeta = 64;  // ints after the list: meta[0, 2 kMaxClasses), padded to 256 bytes
__device__ __align__(256) int32_t scratch[kNoAllocMaxBatch + kScratchMeta];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch[kMaxDevices] = {};

// The device address of this device's scratch array (the current device
// must be h->device).
hipError_t lookup_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  LUPP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = (int32_t*)ptr;
  return hipSuccess;
}

// The class list of an allocating call: grown on demand (this synchronizes
// the handle's streams and reallocates).
hipError_t ensure_batch_list(lupp_handle_t h, int64_t batch) {
  BatchWs* w = h->batch;
  if (!w) return hipErrorNotInitialized;
  if (batch <= w->capacity && w->list) return hipSuccess;
  LUPP_TRY(hipStreamSynchronize(h->stream));
  for (int c = 0; c < kMaxClasses; ++c)
    if (w->streams[c]) LUPP_TRY(hipStreamSynchronize(w->streams[c]));
  if (w->list) (void)hipFree(w->list);
  w->list = nullptr;
  w->capacity = 0;
  const int64_t cap = batch < 1024 ? 1024 : batch;
  void* p = nullptr;
  LUPP_TRY(hipMalloc(&p, (size_t)cap * 4 + 256));
  w->list = (int32_t*)p;
  w->meta = (int32_t*)((char*)p + (size_t)cap * 4);
  w->capacity = cap;
  return hipSuccess;
}

// Binning and the per-class launches on the handle's class streams (forked
// from and joined to the handle's stream), with the class list and counters
// at list / meta.  Launches only: no allocation, no host synchronization.
// The class streams and their events, once per handle (no device memory).
hipError_t ensure_class_streams(BatchWs* w) {
  if (w->fork) return hipSuccess;
  for (int c = 0; c < kMaxClasses; ++c) {
    LUPP_TRY(hipStreamCreateWithFlags(&w->streams[c], hipStreamNonBlocking));
    LUPP_TRY(hipEventCreateWithFlags(&w->join[c], hipEventDisableTiming));
  }
  return hipEventCreateWithFlags(&w->fork, hipEventDisableTiming);
}

template <typename T>
int launch_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* aoff, T* A, const int64_t* poff,
                   int32_t* piv, const int64_t* boff, T* B, int32_t* info, int32_t* list, int32_t* meta) {
  BatchWs* w = h->batch;
  hipStream_t s = h->stream;
  {
    const hipError_t es = ensure_class_streams(w);
    if (es != hipSuccess) return hip_status(es);
  }
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const Schedule& sc = w->sched[prec];
  ClassBounds cb{};
  cb.nclass = sc.nclass;
  for (int c = 0; c < kMaxClasses; ++c) cb.ub[c] = c < sc.nclass ? sc.ub[c] : kBatchMaxN;
  hipLaunchKernelGGL(k_batch_bin, dim3(1), dim3(1024), 0, s, batch, dn, list, meta, info, cb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e);
  e = hipEventRecord(w->fork, s);
  if (e != hipSuccess) return hip_status(e);
  // largest class first: it holds most of the work
  for (int c = sc.nclass - 1; c >= 0; --c) {
    hipStream_t st = w->streams[c];
    e = hipStreamWaitEvent(st, w->fork, 0);
    if (e != hipSuccess) return hip_status(e);
    const int v = sc.shape[c];
    const void* f = shape_kernel<T>(v);
    const int32_t* cmeta = meta;
    const int32_t* clist = list;
    void* args[] = {(void*)&c, (void*)&dn, (void*)&aoff, (void*)&A, (void*)&poff, (void*)&piv, (void*)&boff,
                    (void*)&B, (void*)&info, (void*)&clist, (void*)&cmeta};
    int grid = (int)((int64_t)w->occ[prec][v] * sc.grid_pct[c] / 100);
    if (grid < 1) grid = 1;
    e = hipLaunchKernel(f, dim3(grid), dim3(shape_threads(v)), args, 0, st);
    if (e != hipSuccess) return hip_status(e);
    e = hipEventRecord(w->join[c], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, w->join[c], 0);
    if (e != hipSuccess) return hip_status(e);
  }
  return LUPP_OK;
}

template <typename T>
int gesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* aoff, T* A, const int64_t* poff,
                 int32_t* piv, const int64_t* boff, T* B, int32_t* info) {
  hipError_t e = ensure_batch_list(h, batch);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? LUPP_ERR_ALLOC : hip_status(e);
  return launch_batched<T>(h, batch, dn, aoff, A, poff, piv, boff, B, info, h->batch->list, h->batch->meta);
}

}  // namespace

// At handle creation, on the handle's device: the persistent grids, the
// schedules, and the device address of the scratch array.  No device memory
// is allocated here; the class streams are created by the first batched call
// (ensure_class_streams), so that a handle that never runs the batched path
// holds no streams for it.
hipError_t setup_batched(lupp_handle_t h) {
  LUPP_TRY(lookup_scratch(h->device));
  BatchWs* w = new (std::nothrow) BatchWs();
  if (!w) return hipErrorOutOfMemory;
  h->batch = w;
  LUPP_TRY(setup_shape_occupancy<double>(h, w, 0));
  LUPP_TRY(setup_shape_occupancy<float>(h, w, 1));
  w->sched[0] = default_schedule(0);
  w->sched[1] = default_schedule(1);
  return hipSuccess;
}

namespace {

template <typename T>
int batched_entry(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* aoff, T* A,
                  const int64_t* poff, int32_t* piv, const int64_t* boff, T* B, int32_t* info, bool solve) {
  if (!h) return -1;
  if (batch < 0) return -2;
  if (batch == 0) return LUPP_OK;
  if (!dn) return -3;
  if (!aoff) return -4;
  if (!A) return -5;
  if (!poff) return -6;
  if (!piv) return -7;
  if (solve && !boff) return -8;
  if (solve && !B) return -9;
  if (!info) return solve ? -10 : -8;
  return gesv_batched<T>(h, batch, dn, aoff, A, poff, piv, solve ? boff : nullptr, solve ? B : nullptr, info);
}

}  // namespace
}  // namespace lupp

extern "C" {

int lupp_batched_shape(int32_t v, int32_t* nw, int32_t* rows, int32_t* cols, int32_t* nmax) {
  if (v < 0 || v >= lupp::kNumShapes) return -1;
  if (nw) *nw = lupp::kShapes[v].nw;
  if (rows) *rows = 64 * lupp::kShapes[v].r;
  if (cols) *cols = lupp::kShapes[v].c;
  if (nmax) *nmax = lupp::shape_nmax(v);
  return LUPP_OK;
}

int lupp_batched_shape_count(void) { return lupp::kNumShapes; }

namespace {
void to_c(const lupp::Schedule& s, lupp_batched_schedule* o) {
  *o = lupp_batched_schedule{};
  o->nclass = s.nclass;
  for (int c = 0; c < s.nclass; ++c) {
    o->nmax[c] = s.ub[c];
    o->shape[c] = s.shape[c];
    o->grid_pct[c] = s.grid_pct[c];
  }
}
}  // namespace

int lupp_batched_get_schedule(lupp_handle_t h, int32_t fp32, lupp_batched_schedule* out) {
  if (!h) return -1;
  if (fp32 != 0 && fp32 != 1) return -2;
  if (!out) return -3;
  if (!h->batch) return LUPP_ERR_INTERNAL;
  to_c(h->batch->sched[fp32], out);
  return LUPP_OK;
}

int lupp_batched_set_schedule(lupp_handle_t h, int32_t fp32, const lupp_batched_schedule* s) {
  if (!h) return -1;
  if (fp32 != 0 && fp32 != 1) return -2;
  if (!h->batch) return LUPP_ERR_INTERNAL;
  if (!s) {
    h->batch->sched[fp32] = lupp::default_schedule(fp32);
    return LUPP_OK;
  }
  lupp::Schedule t;
  t.nclass = s->nclass;
  if (t.nclass < 1 || t.nclass > lupp::kMaxClasses) return -3;
  for (int c = 0; c < t.nclass; ++c) {
    t.ub[c] = s->nmax[c];
    t.shape[c] = s->shape[c];
    t.grid_pct[c] = s->grid_pct[c];
  }
  if (!lupp::schedule_valid(t)) return -3;
  h->batch->sched[fp32] = t;
  return LUPP_OK;
}

int lupp_dgesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off, double* dA,
                       const int64_t* dipiv_off, int32_t* dipiv, const int64_t* dB_off, double* dB,
                       int32_t* dinfo) {
  return lupp::batched_entry<double>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, dB_off, dB, dinfo, true);
}

int lupp_sgesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off, float* dA,
                       const int64_t* dipiv_off, int32_t* dipiv, const int64_t* dB_off, float* dB,
                       int32_t* dinfo) {
  return lupp::batched_entry<float>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, dB_off, dB, dinfo, true);
}

int lupp_dgetrf_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off, double* dA,
                        const int64_t* dipiv_off, int32_t* dipiv, int32_t* dinfo) {
  return lupp::batched_entry<double>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, nullptr, nullptr, dinfo, false);
}

int lupp_dgesv_batched_noalloc(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off,
                                double* dA, const int64_t* dipiv_off, int32_t* dipiv, const int64_t* dB_off,
                                double* dB, int32_t* dinfo) {
  if (!h) return -1;
  if (batch < 0) return -2;
  if (batch > lupp::kNoAllocMaxBatch) return LUPP_ERR_UNSUPPORTED;
  if (batch == 0) return LUPP_OK;
  if (!dn) return -3;
  if (!dA_off) return -4;
  if (!dA) return -5;
  if (!dipiv_off) return -6;
  if (!dipiv) return -7;
  if (!dB_off) return -8;
  if (!dB) return -9;
  if (!dinfo) return -10;
  if (!h->batch || h->device < 0 || h->device >= lupp::kMaxDevices) return LUPP_ERR_INTERNAL;
  int32_t* list = lupp::g_scratch[h->device];
  if (!list) return LUPP_ERR_INTERNAL;
  return lupp::launch_batched<double>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, dB_off, dB, dinfo, list,
                                      list + lupp::kNoAllocMaxBatch);
}

int lupp_sgetrf_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off, float* dA,
                        const int64_t* dipiv_off, int32_t* dipiv, int32_t* dinfo) {
  return lupp::batched_entry<float>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, nullptr, nullptr, dinfo, false);
}

}  // extern "C"
