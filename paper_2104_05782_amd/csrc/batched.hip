// Batched LU with partial pivoting and solve for many small systems
// (order n <= 128), one workgroup per system with the system held in LDS.
//
// Each system is the same factorization as the large path -- partial
// pivoting with LAPACK's conventions, blocked right-looking with a W-column
// panel and a rank-W trailing update (the blocked loop of Section 4.3 and
// the column-block step of Section 4.1, at the scale of one workgroup) --
// applied to the augmented matrix [A | b], so that the row interchanges and
// the elimination also carry b to L^{-1} P b; a backward substitution with U
// then gives x (skipped, as in LAPACK's gesv, when a pivot is exactly zero).
//
// Scheduling: a binning kernel sorts the systems into four size classes
// (n <= 32, 64, 96, 128), each served by one persistent launch whose
// workgroups (64, 256, 512, 512 threads) take systems from an atomic queue;
// the LDS footprint of a class is its largest augmented matrix, so smaller
// classes run more workgroups per CU.  The classes are launched on four
// streams so that the short classes fill the CUs the long ones leave idle.
// No host synchronization or allocation happens per call (graph-capturable
// once the workspace exists for the batch size).
#include "handle.h"
#include "wave.h"

namespace lupp {

constexpr int kBatchClasses = 4;
constexpr int kBatchMaxN = 128;

// Workspace of the batched path: per-class system lists and counters.
struct BatchWs {
  int64_t capacity = 0;
  int32_t* list = nullptr;  // capacity entries: system ids grouped by class
  int32_t* meta = nullptr;  // [0,4) counts, [4,8) offsets, [8,12) queue heads
  hipStream_t streams[kBatchClasses] = {};
  hipEvent_t fork = nullptr, join[kBatchClasses] = {};
  int grid[2][kBatchClasses] = {};  // persistent grid per (precision, class)
};

namespace {

constexpr int kPanelW = 8;  // panel width of the per-system blocked factorization

__device__ __forceinline__ int size_class(int n) { return n <= 32 ? 0 : (n <= 64 ? 1 : (n <= 96 ? 2 : 3)); }

// Sort systems into size classes; reset the queue heads.  One workgroup.
__global__ __launch_bounds__(1024) void k_batch_bin(int32_t batch, const int32_t* __restrict__ dn,
                                                    int32_t* __restrict__ list, int32_t* __restrict__ meta,
                                                    int32_t* __restrict__ info) {
  __shared__ int cnt[kBatchClasses], cur[kBatchClasses], off[kBatchClasses];
  const int tid = threadIdx.x;
  if (tid < kBatchClasses) cnt[tid] = 0;
  __syncthreads();
  for (int i = tid; i < batch; i += 1024) {
    const int n = dn[i];
    if (n >= 1 && n <= kBatchMaxN) atomicAdd(&cnt[size_class(n)], 1);
    else info[i] = (n == 0) ? 0 : -1;  // empty system: nothing to do; bad order: rejected
  }
  __syncthreads();
  if (tid == 0) {
    int o = 0;
    for (int c = 0; c < kBatchClasses; ++c) {
      off[c] = o;
      cur[c] = 0;
      meta[c] = cnt[c];
      meta[4 + c] = o;
      meta[8 + c] = 0;
      o += cnt[c];
    }
  }
  __syncthreads();
  for (int i = tid; i < batch; i += 1024) {
    const int n = dn[i];
    if (n >= 1 && n <= kBatchMaxN) {
      const int c = size_class(n);
      list[off[c] + atomicAdd(&cur[c], 1)] = i;
    }
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_batch_lu(int cls, const int32_t* __restrict__ dn,
                                                 const int64_t* __restrict__ aoff, T* __restrict__ gA,
                                                 const int64_t* __restrict__ poff, int32_t* __restrict__ gpiv,
                                                 const int64_t* __restrict__ boff, T* __restrict__ gB,
                                                 int32_t* __restrict__ ginfo, const int32_t* __restrict__ list,
                                                 int32_t* __restrict__ meta) {
  constexpr int NW = NT / 64;
  constexpr int W = kPanelW;
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  T* As = (T*)dyn;  // n x (n + 1), leading dimension n
  __shared__ int s_piv[kBatchMaxN];
  __shared__ int s_pdst[2 * W], s_psrc[2 * W];
  __shared__ int s_sys, s_info, s_npairs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int count = meta[cls], first = meta[4 + cls];

  for (;;) {
    if (tid == 0) {
      const int q = atomicAdd(&meta[8 + cls], 1);
      s_sys = q < count ? list[first + q] : -1;
      s_info = 0;
    }
    __syncthreads();
    const int sys = s_sys;
    if (sys < 0) return;
    const int n = dn[sys];
    T* A = gA + aoff[sys];
    T* Bv = gB ? gB + boff[sys] : nullptr;
    const int ncol = n + (Bv ? 1 : 0);
    const int nn = n * n;
    // ---- system into LDS, eight loads in flight per thread
    for (int base = 0; base < nn; base += 8 * NT) {
      T tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT + tid;
        tmp[u] = (e < nn) ? A[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT + tid;
        if (e < nn) As[e] = tmp[u];
      }
    }
    if (Bv)
      for (int i = tid; i < n; i += NT) As[nn + i] = Bv[i];
    __syncthreads();

    for (int j0 = 0; j0 < n; j0 += W) {
      const int w = (n - j0 < W) ? (n - j0) : W;
      // ---- panel: columns j0 .. j0+w-1, rows j0 .. n-1, factored by wave 0
      // with the rows in registers (lane holds rows lane and lane + 64).  Rows
      // are not moved during the panel: pos0/pos1 give the logical row whose
      // data each slot holds, an interchange swaps two logical positions, and
      // the data is written to its final rows once at the end.
      if (wave == 0) {
        const int r0 = lane, r1 = lane + 64;
        const bool ok0 = r0 >= j0 && r0 < n, ok1 = r1 >= j0 && r1 < n;
        int pos0 = r0, pos1 = r1;
        T v0[W], v1[W];
#pragma unroll
        for (int t = 0; t < W; ++t) {
          v0[t] = (t < w && ok0) ? As[r0 + (j0 + t) * n] : T(0);
          v1[t] = (t < w && ok1) ? As[r1 + (j0 + t) * n] : T(0);
        }
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (t < w) {
            const int c = j0 + t;
            // pivot: the largest |a| over logical rows >= c, lowest row on ties
            const bool q0 = ok0 && pos0 >= c, q1 = ok1 && pos1 >= c;
            const double a0 = q0 ? (double)fabs(v0[t]) : -1.0, a1 = q1 ? (double)fabs(v1[t]) : -1.0;
            const double m = wave_max_f64(fmax(a0, a1));
            const uint32_t k0 = (q0 && a0 == m) ? (uint32_t)pos0 : 0x7fffffffu;
            const uint32_t k1 = (q1 && a1 == m) ? (uint32_t)pos1 : 0x7fffffffu;
            const uint32_t pm = wave_min_u32(min(k0, k1));
            const int p = (pm >= (uint32_t)c && pm < (uint32_t)n) ? (int)pm : c;  // c only with NaN entries
            // where logical row p lives
            const uint64_t b0 = __ballot(ok0 && pos0 == p), b1 = __ballot(ok1 && pos1 == p);
            const bool in1 = b0 == 0;
            const uint64_t bm = in1 ? b1 : b0;
            const int pl = bm ? (int)__builtin_ctzll(bm) : 0;
            T rp[W];
#pragma unroll
            for (int t2 = 0; t2 < W; ++t2) {
              rp[t2] = T(0);
              if (t2 >= t && t2 < w) rp[t2] = readlane_d(in1 ? v1[t2] : v0[t2], pl);
            }
            const T pv = rp[t];
            if (lane == 0) {
              s_piv[c] = p;
              if (pv == T(0) && s_info == 0) s_info = c + 1;
            }
            if (p != c) {
              pos0 = (pos0 == c) ? p : ((pos0 == p) ? c : pos0);
              pos1 = (pos1 == c) ? p : ((pos1 == p) ? c : pos1);
            }
            // multipliers (true division: |l| <= 1 exactly) and the panel's rank-1 update
            if (pv != T(0)) {
              if (ok0 && pos0 > c) {
                const T l = v0[t] / pv;
                v0[t] = l;
#pragma unroll
                for (int t2 = t + 1; t2 < W; ++t2) v0[t2] -= l * rp[t2];
              }
              if (ok1 && pos1 > c) {
                const T l = v1[t] / pv;
                v1[t] = l;
#pragma unroll
                for (int t2 = t + 1; t2 < W; ++t2) v1[t2] -= l * rp[t2];
              }
            }
          }
        }
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (t < w && ok0) As[pos0 + (j0 + t) * n] = v0[t];
          if (t < w && ok1) As[pos1 + (j0 + t) * n] = v1[t];
        }
        // the block's interchanges composed: row pos <- row r for every moved row
        const bool mv0 = ok0 && pos0 != r0, mv1 = ok1 && pos1 != r1;
        const uint64_t m0 = __ballot(mv0), m1 = __ballot(mv1);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int cnt0 = __popcll(m0);
        if (mv0) {
          const int q = __popcll(m0 & below);
          s_pdst[q] = pos0;
          s_psrc[q] = r0;
        }
        if (mv1) {
          const int q = cnt0 + __popcll(m1 & below);
          s_pdst[q] = pos1;
          s_psrc[q] = r1;
        }
        if (lane == 0) s_npairs = cnt0 + __popcll(m1);
      }
      __syncthreads();
      // ---- per column outside the panel (b included), one column per thread:
      // the block's composed interchanges (all moved rows read, then
      // written), then U12 := inv(L11) A12 for the columns right of the panel
      const int j1 = j0 + w;
      {
        const int np = s_npairs;
        for (int j = tid; j < ncol; j += NT) {
          if (j >= j0 && j < j1) continue;
          if (np > 0) {
            T val[2 * W];
#pragma unroll
            for (int q = 0; q < 2 * W; ++q)
              if (q < np) val[q] = As[s_psrc[q] + j * n];
#pragma unroll
            for (int q = 0; q < 2 * W; ++q)
              if (q < np) As[s_pdst[q] + j * n] = val[q];
          }
          if (j >= j1) {
            T x[W];
#pragma unroll
            for (int q = 0; q < W; ++q) x[q] = (q < w) ? As[j0 + q + j * n] : T(0);
#pragma unroll
            for (int q = 0; q < W; ++q)
#pragma unroll
              for (int r = q + 1; r < W; ++r)
                if (r < w) x[r] -= As[j0 + r + (j0 + q) * n] * x[q];
#pragma unroll
            for (int q = 1; q < W; ++q)
              if (q < w) As[j0 + q + j * n] = x[q];
          }
        }
      }
      if (j1 >= ncol) break;
      __syncthreads();
      // ---- A22 -= L21 U12: lanes over rows (two 64-row halves), waves over
      // columns, two columns per step
      if (j1 < n) {
        T l[2][W];
        const int i0 = j1 + lane, i1 = j1 + 64 + lane;
#pragma unroll
        for (int q = 0; q < W; ++q) {
          l[0][q] = (q < w && i0 < n) ? As[i0 + (j0 + q) * n] : T(0);
          l[1][q] = (q < w && i1 < n) ? As[i1 + (j0 + q) * n] : T(0);
        }
        for (int j = j1 + wave; j < ncol; j += 2 * NW) {
          const int jb = j + NW;
          const bool two = jb < ncol;
          T u[W], ub[W];
#pragma unroll
          for (int q = 0; q < W; ++q) {
            u[q] = (q < w) ? As[j0 + q + j * n] : T(0);
            ub[q] = (q < w && two) ? As[j0 + q + jb * n] : T(0);
          }
          T s0 = (i0 < n) ? As[i0 + j * n] : T(0);
          T s1 = (i1 < n) ? As[i1 + j * n] : T(0);
          T s2 = (i0 < n && two) ? As[i0 + jb * n] : T(0);
          T s3 = (i1 < n && two) ? As[i1 + jb * n] : T(0);
#pragma unroll
          for (int q = 0; q < W; ++q) {
            s0 -= l[0][q] * u[q];
            s1 -= l[1][q] * u[q];
            s2 -= l[0][q] * ub[q];
            s3 -= l[1][q] * ub[q];
          }
          if (i0 < n) As[i0 + j * n] = s0;
          if (i1 < n) As[i1 + j * n] = s1;
          if (two && i0 < n) As[i0 + jb * n] = s2;
          if (two && i1 < n) As[i1 + jb * n] = s3;
        }
      }
      __syncthreads();
    }
    __syncthreads();

    // ---- x = inv(U) c with c = L^{-1} P b in column n (one wave; skipped on a
    // zero pivot, as in LAPACK's gesv): reciprocals of the diagonal first, the
    // next column of U prefetched while the current one is applied
    const int info = s_info;
    if (Bv && info == 0 && wave == 0) {
      T c0 = (lane < n) ? As[nn + lane] : T(0);
      T c1 = (lane + 64 < n) ? As[nn + lane + 64] : T(0);
      const T d0 = (lane < n) ? T(1) / As[lane + lane * n] : T(0);
      const T d1 = (lane + 64 < n) ? T(1) / As[lane + 64 + (lane + 64) * n] : T(0);
      int k = n - 1;
      T u0 = (lane < k) ? As[lane + k * n] : T(0);
      T u1 = (lane + 64 < k) ? As[lane + 64 + k * n] : T(0);
      for (; k >= 0; --k) {
        T u0n = T(0), u1n = T(0);
        if (k > 0) {
          if (lane < k - 1) u0n = As[lane + (k - 1) * n];
          if (lane + 64 < k - 1) u1n = As[lane + 64 + (k - 1) * n];
        }
        const bool hi = k >= 64;
        const int kl = hi ? k - 64 : k;
        const T xk = readlane_d(hi ? c1 : c0, kl) * readlane_d(hi ? d1 : d0, kl);
        if (!hi && lane == kl) c0 = xk;
        if (hi && lane == kl) c1 = xk;
        c0 -= u0 * xk;
        c1 -= u1 * xk;
        u0 = u0n;
        u1 = u1n;
      }
      if (lane < n) Bv[lane] = c0;
      if (lane + 64 < n) Bv[lane + 64] = c1;
    }
    for (int e = tid; e < nn; e += NT) A[e] = As[e];
    int32_t* P = gpiv + poff[sys];
    for (int k = tid; k < n; k += NT) P[k] = s_piv[k] + 1;
    if (tid == 0) ginfo[sys] = info;
    __syncthreads();
  }
}

template <typename T>
const void* batch_kernel(int cls) {
  switch (cls) {
    case 0: return (const void*)k_batch_lu<T, 64>;
    case 1: return (const void*)k_batch_lu<T, 256>;
    default: return (const void*)k_batch_lu<T, 512>;
  }
}
inline int class_threads(int cls) { return cls == 0 ? 64 : (cls == 1 ? 256 : 512); }
inline int class_nmax(int cls) { return 32 * (cls + 1); }
template <typename T>
size_t class_lds(int cls) {
  const size_t nm = (size_t)class_nmax(cls);
  return nm * (nm + 1) * sizeof(T);
}

template <typename T>
hipError_t setup_class_kernels(lupp_handle_t h, BatchWs* w, int prec) {
  int ncu = 0;
  LUPP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
  for (int c = 0; c < kBatchClasses; ++c) {
    const void* f = batch_kernel<T>(c);
    const size_t lds = class_lds<T>(c);
    LUPP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int occ = 0;
    LUPP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, class_threads(c), lds));
    if (occ < 1) return hipErrorInvalidConfiguration;
    w->grid[prec][c] = occ * ncu;
  }
  return hipSuccess;
}

}  // namespace

void free_batched(lupp_handle_t h) {
  BatchWs* w = h->batch;
  if (!w) return;
  for (int c = 0; c < kBatchClasses; ++c) {
    if (w->streams[c]) (void)hipStreamSynchronize(w->streams[c]);
    if (w->join[c]) (void)hipEventDestroy(w->join[c]);
    if (w->streams[c]) (void)hipStreamDestroy(w->streams[c]);
  }
  if (w->fork) (void)hipEventDestroy(w->fork);
  if (w->list) (void)hipFree(w->list);
  delete w;
  h->batch = nullptr;
}

namespace {

hipError_t ensure_batch(lupp_handle_t h, int64_t batch) {
  BatchWs* w = h->batch;
  if (!w) {
    w = new (std::nothrow) BatchWs();
    if (!w) return hipErrorOutOfMemory;
    h->batch = w;
    for (int c = 0; c < kBatchClasses; ++c) {
      LUPP_TRY(hipStreamCreateWithFlags(&w->streams[c], hipStreamNonBlocking));
      LUPP_TRY(hipEventCreateWithFlags(&w->join[c], hipEventDisableTiming));
    }
    LUPP_TRY(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
    LUPP_TRY(setup_class_kernels<double>(h, w, 0));
    LUPP_TRY(setup_class_kernels<float>(h, w, 1));
  }
  if (batch <= w->capacity && w->list) return hipSuccess;
  LUPP_TRY(hipStreamSynchronize(h->stream));
  for (int c = 0; c < kBatchClasses; ++c) LUPP_TRY(hipStreamSynchronize(w->streams[c]));
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

template <typename T>
int gesv_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* aoff, T* A, const int64_t* poff,
                 int32_t* piv, const int64_t* boff, T* B, int32_t* info) {
  hipError_t e = ensure_batch(h, batch);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? LUPP_ERR_ALLOC : hip_status(e);
  BatchWs* w = h->batch;
  hipStream_t s = h->stream;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  hipLaunchKernelGGL(k_batch_bin, dim3(1), dim3(1024), 0, s, batch, dn, w->list, w->meta, info);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e);
  e = hipEventRecord(w->fork, s);
  if (e != hipSuccess) return hip_status(e);
  // largest class first: it holds most of the work
  for (int c = kBatchClasses - 1; c >= 0; --c) {
    hipStream_t sc = w->streams[c];
    e = hipStreamWaitEvent(sc, w->fork, 0);
    if (e != hipSuccess) return hip_status(e);
    const void* f = batch_kernel<T>(c);
    void* args[] = {(void*)&c, (void*)&dn, (void*)&aoff, (void*)&A, (void*)&poff, (void*)&piv, (void*)&boff,
                    (void*)&B, (void*)&info, (void*)&w->list, (void*)&w->meta};
    e = hipLaunchKernel(f, dim3(w->grid[prec][c]), dim3(class_threads(c)), args, class_lds<T>(c), sc);
    if (e != hipSuccess) return hip_status(e);
    e = hipEventRecord(w->join[c], sc);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, w->join[c], 0);
    if (e != hipSuccess) return hip_status(e);
  }
  return LUPP_OK;
}

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

int lupp_sgetrf_batched(lupp_handle_t h, int32_t batch, const int32_t* dn, const int64_t* dA_off, float* dA,
                        const int64_t* dipiv_off, int32_t* dipiv, int32_t* dinfo) {
  return lupp::batched_entry<float>(h, batch, dn, dA_off, dA, dipiv_off, dipiv, nullptr, nullptr, dinfo, false);
}

}  // extern "C"
