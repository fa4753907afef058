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
// workgroups (64, 128, 256, 256 threads) take systems from an atomic queue;
// the LDS footprint of a class is its largest augmented matrix, so smaller
// classes run more workgroups per CU.  The classes are launched on four
// streams so that the short classes fill the CUs the long ones leave idle.
// No host synchronization or allocation happens per call (graph-capturable
// once the workspace exists for the batch size).
#include "handle.h"

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

__device__ __forceinline__ double readlane_d(double v, int k) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float readlane_d(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

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

// (|v|, row) argmax with the lowest row among equal magnitudes
template <typename T>
__device__ __forceinline__ void better_of(T& av, int& ai, T& sv, T bv, int bi, T bs) {
  if (bv > av || (bv == av && bi < ai)) {
    av = bv;
    ai = bi;
    sv = bs;
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
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  T* As = (T*)dyn;  // n x (n + 1), leading dimension n
  __shared__ T s_wabs[NW], s_wval[NW];
  __shared__ int s_widx[NW];
  __shared__ int s_piv[kBatchMaxN];
  __shared__ int s_sys, s_info;
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
    for (int e = tid; e < nn; e += NT) As[e] = A[e];
    if (Bv)
      for (int i = tid; i < n; i += NT) As[nn + i] = Bv[i];
    __syncthreads();

    for (int j0 = 0; j0 < n; j0 += kPanelW) {
      const int w = (n - j0 < kPanelW) ? (n - j0) : kPanelW;
      // ---- panel: columns j0 .. j0+w-1, rows j0 .. n-1
      for (int t = 0; t < w; ++t) {
        const int c = j0 + t;
        T av = T(-1), sv = T(0);
        int ai = 0x7fffffff;
        if (tid >= c && tid < n) {
          sv = As[tid + c * n];
          av = fabs(sv);
          ai = tid;
        }
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
          const T bv = __shfl_xor(av, m, 64);
          const int bi = __shfl_xor(ai, m, 64);
          const T bs = __shfl_xor(sv, m, 64);
          better_of(av, ai, sv, bv, bi, bs);
        }
        if (lane == 0) {
          s_wabs[wave] = av;
          s_wval[wave] = sv;
          s_widx[wave] = ai;
        }
        __syncthreads();
        T pa = s_wabs[0], pv = s_wval[0];
        int p = s_widx[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) better_of(pa, p, pv, s_wabs[q], s_widx[q], s_wval[q]);
        if (p < c || p >= n) p = c;  // only reachable with NaN entries (outside the contract)
        if (tid == 0) {
          s_piv[c] = p;
          if (pv == T(0) && s_info == 0) s_info = c + 1;
        }
        // interchange rows c and p in every column (b included); one column per thread
        if (p != c && tid < ncol) {
          const T x = As[c + tid * n];
          As[c + tid * n] = As[p + tid * n];
          As[p + tid * n] = x;
        }
        __syncthreads();
        // multipliers of column c and their update of the rest of the panel
        if (pv != T(0) && tid > c && tid < n) {
          const T l = As[tid + c * n] / pv;
          As[tid + c * n] = l;
          for (int t2 = t + 1; t2 < w; ++t2) {
            const int col = j0 + t2;
            As[tid + col * n] -= l * As[c + col * n];
          }
        }
        __syncthreads();
      }
      const int j1 = j0 + w;
      if (j1 >= ncol) break;
      // ---- U12 := inv(L11) A12 (rows j0..j1-1, columns j1..ncol-1), one column per thread
      for (int j = j1 + tid; j < ncol; j += NT) {
        T x[kPanelW];
#pragma unroll
        for (int r = 0; r < kPanelW; ++r) x[r] = (r < w) ? As[j0 + r + j * n] : T(0);
#pragma unroll
        for (int r = 1; r < kPanelW; ++r) {
          if (r < w) {
            T s = x[r];
#pragma unroll
            for (int q = 0; q < kPanelW; ++q)
              if (q < r) s -= As[j0 + r + (j0 + q) * n] * x[q];
            x[r] = s;
          }
        }
#pragma unroll
        for (int r = 1; r < kPanelW; ++r)
          if (r < w) As[j0 + r + j * n] = x[r];
      }
      __syncthreads();
      // ---- A22 -= L21 U12: lanes over rows (two 64-row halves), waves over columns
      if (j1 < n) {
        T l[2][kPanelW];
        const int i0 = j1 + lane, i1 = j1 + 64 + lane;
#pragma unroll
        for (int q = 0; q < kPanelW; ++q) {
          l[0][q] = (q < w && i0 < n) ? As[i0 + (j0 + q) * n] : T(0);
          l[1][q] = (q < w && i1 < n) ? As[i1 + (j0 + q) * n] : T(0);
        }
        for (int j = j1 + wave; j < ncol; j += NW) {
          T u[kPanelW];
#pragma unroll
          for (int q = 0; q < kPanelW; ++q) u[q] = (q < w) ? As[j0 + q + j * n] : T(0);
          if (i0 < n) {
            T s = As[i0 + j * n];
#pragma unroll
            for (int q = 0; q < kPanelW; ++q) s -= l[0][q] * u[q];
            As[i0 + j * n] = s;
          }
          if (i1 < n) {
            T s = As[i1 + j * n];
#pragma unroll
            for (int q = 0; q < kPanelW; ++q) s -= l[1][q] * u[q];
            As[i1 + j * n] = s;
          }
        }
      }
      __syncthreads();
    }

    // ---- x = inv(U) c, c = L^{-1} P b in column n (one wave; skipped on a zero pivot)
    const int info = s_info;
    if (Bv && info == 0 && wave == 0) {
      T c0 = (lane < n) ? As[nn + lane] : T(0);
      T c1 = (lane + 64 < n) ? As[nn + lane + 64] : T(0);
      for (int k = n - 1; k >= 0; --k) {
        const T ck = (k < 64) ? readlane_d(c0, k) : readlane_d(c1, k - 64);
        const T xk = ck / As[k + k * n];
        if (k < 64) {
          if (lane == k) c0 = xk;
        } else {
          if (lane == k - 64) c1 = xk;
        }
        if (lane < k) c0 -= As[lane + k * n] * xk;
        if (lane + 64 < k) c1 -= As[lane + 64 + k * n] * xk;
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
    case 1: return (const void*)k_batch_lu<T, 128>;
    default: return (const void*)k_batch_lu<T, 256>;
  }
}
inline int class_threads(int cls) { return cls == 0 ? 64 : (cls == 1 ? 128 : 256); }
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
