// Kernels of the solve and of the FP64 iterative refinement.
//
// * k_trsv: one-launch triangular solve for one right-hand side.  The n rows
//   are cut into 64-row blocks; each workgroup takes the next block in
//   dispatch order (a ticket from an atomic counter, so every block it waits
//   for was dispatched before it), subtracts the contributions of the finished
//   blocks as their flags appear (it polls 64 flags per load), solves its
//   diagonal block inside one wavefront (lane i holds row i of the block in
//   registers; x_k is read with readlane), and publishes its x with
//   device-coherent stores before raising its flag.  The matrix is read once.
// * k_trsv128: the same chain over 128-row blocks (eight wavefronts, two
//   64-row diagonal solves with the off-diagonal 64x64 update between them),
//   used from kTrsvWideMinN rows on: half as many handoffs between workgroups.
// * k_gemv_part / k_gemv_fin: r = b - A x in FP64, two passes over column
//   chunks, deterministic (no floating-point atomics).
// * norms, dot products, axpy and format conversions for the refinement.
#include "common.h"

namespace lupp {
namespace {

constexpr int TB = 64;                // rows per triangular-solve block
constexpr int TB2 = 128;              // rows per block of the wide variant
constexpr int64_t kTrsvWideMinN = 8192;  // the wide variant from this order on

__device__ __forceinline__ double readlane_t(double v, int k) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float readlane_t(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v);
template <>
__device__ __forceinline__ void st_coh<double>(double* p, double v) {
  __hip_atomic_store((uint64_t*)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <>
__device__ __forceinline__ void st_coh<float>(float* p, float v) {
  __hip_atomic_store((uint32_t*)p, __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_coh(const T* p);
template <>
__device__ __forceinline__ double ld_coh<double>(const double* p) {
  return __longlong_as_double(
      (long long)__hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <>
__device__ __forceinline__ float ld_coh<float>(const float* p) {
  return __uint_as_float(__hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

template <typename T, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(int64_t n, const T* __restrict__ A, int64_t lda, T* __restrict__ x,
                                              uint32_t* __restrict__ flags, uint64_t* __restrict__ ticket,
                                              uint64_t tbase, uint32_t epoch, int32_t* __restrict__ err) {
  __shared__ T s_part[4][TB];
  __shared__ T s_diag[TB * TB];
  __shared__ int64_t s_blk;
  __shared__ int s_ready;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nblk = (n + TB - 1) / TB;
  if (tid == 0) s_blk = (int64_t)(atomicAdd((unsigned long long*)ticket, 1ull) - tbase);
  __syncthreads();
  const int64_t q = s_blk;
  if (q < 0 || q >= nblk) {  // ticket bookkeeping out of step: report, touch nothing
    if (tid == 0) *err = 2;
    return;
  }
  const int64_t b = LOWER ? q : (nblk - 1 - q);
  const int64_t r0 = b * TB;
  const int64_t row = r0 + lane;
  const bool rok = row < n;
  T acc = T(0);
  // dependencies: blocks [0, b) (lower) or (b, nblk) (upper), in order
  const int64_t ndep = LOWER ? b : (nblk - 1 - b);
  // The last dependency (the adjacent block) is on the critical path: its
  // matrix tile does not depend on the flag, so this wave's 16 columns of it
  // are loaded now; after the flag only x is read.
  T apf[16];
  // the diagonal block depends on nothing either: staged in LDS before the
  // waits (column-major, so wave 0 reads its rows without bank conflicts), it
  // is off the critical path
  for (int e = tid; e < TB * TB; e += 256) {
    const int c = e / TB, rr = e % TB;
    s_diag[e] = (r0 + rr < n && r0 + c < n) ? A[(r0 + rr) + (r0 + c) * lda] : T(0);
  }
  const int64_t lastd = ndep - 1;
  if (ndep > 0) {
    const int64_t c0 = (LOWER ? lastd : (nblk - 1 - lastd)) * TB + wave * 16;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int64_t c = c0 + cc;
      apf[cc] = (c < n && rok) ? A[row + c * lda] : T(0);
    }
  }
  int64_t done = 0;
  long spins = 0;
  while (done < ndep) {
    // wave 0 finds how many further blocks are ready
    if (wave == 0) {
      const int64_t d0 = done + lane;
      const int64_t blk = LOWER ? d0 : (nblk - 1 - d0);
      bool ok = true;
      if (d0 < ndep) ok = __hip_atomic_load(&flags[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      const unsigned long long notready = __ballot(!ok);
      const int nready = notready ? (__ffsll((long long)notready) - 1) : 64;
      if (lane == 0) s_ready = nready;
    }
    __syncthreads();
    int nready = s_ready;
    if (nready == 0) {
      if (++spins > (1L << 22)) {
        if (tid == 0) *err = 1;
        nready = (int)(ndep - done);  // give up waiting (results invalid, flagged)
      } else {
        __syncthreads();
        continue;
      }
    }
    for (int64_t d = done; d < done + nready && d < lastd; ++d) {
      const int64_t blk = LOWER ? d : (nblk - 1 - d);
      const int64_t c0 = blk * TB;
      // this wave's 16 columns of the 64x64 tile.  Every load is issued
      // before the first use, so a finished block costs one memory round
      // trip: with four loads in flight at a time the catch-up on each new
      // block took longer than a chain step and set the solve's pace.
      T av[16], xw[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        const int64_t c = c0 + wave * 16 + cc;
        av[cc] = (c < n && rok) ? A[row + c * lda] : T(0);
        xw[cc] = (c < n) ? ld_coh(&x[c]) : T(0);
      }
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc = acc - av[cc] * xw[cc];
    }
    done += nready;
    __syncthreads();
  }
  if (ndep > 0) {
    const int64_t c0 = (LOWER ? lastd : (nblk - 1 - lastd)) * TB + wave * 16;
    T xv[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) xv[cc] = (c0 + cc < n) ? ld_coh(&x[c0 + cc]) : T(0);
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc = acc - apf[cc] * xv[cc];
  }
  s_part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    T v = rok ? x[row] : T(0);
    v = v + s_part[0][lane] + s_part[1][lane] + s_part[2][lane] + s_part[3][lane];
    // diagonal block (staged at the start): lane holds row `lane` of it
    T dr[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) dr[c] = s_diag[c * TB + lane];
    if (LOWER) {
#pragma unroll
      for (int k = 0; k < TB; ++k) {
        const T xk = readlane_t(v, k);
        if (lane > k) v = v - dr[k] * xk;
      }
    } else {
      // each lane's reciprocal of its diagonal entry, computed once: the
      // chain below then multiplies instead of dividing (64 dependent
      // divisions were half of the upper solve's step)
      const T dinv = T(1) / s_diag[lane * TB + lane];
#pragma unroll
      for (int k = TB - 1; k >= 0; --k) {
        if (lane == k && rok) v = v * dinv;
        const T xk = readlane_t(v, k);
        if (lane < k) v = v - dr[k] * xk;
      }
    }
    if (rok) st_coh(&x[row], v);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (lane == 0) __hip_atomic_store(&flags[b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// x := inverse of one 64x64 diagonal block (unit lower, or upper with its
// diagonal) times v; lane i holds row i; sd is the block, column-major in LDS
template <typename T, bool LOWER>
__device__ __forceinline__ T solve64(T v, const T* __restrict__ sd, int lane, bool rok) {
  T dr[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) dr[c] = sd[c * 64 + lane];
  if (LOWER) {
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const T xk = readlane_t(v, k);
      if (lane > k) v = v - dr[k] * xk;
    }
  } else {
    const T dinv = T(1) / sd[lane * 64 + lane];
#pragma unroll
    for (int k = 63; k >= 0; --k) {
      if (lane == k && rok) v = v * dinv;
      const T xk = readlane_t(v, k);
      if (lane < k) v = v - dr[k] * xk;
    }
  }
  return v;
}

// 128-row blocks: wavefront w covers rows 64*(w/4) .. +63 of the block and
// columns 32*(w%4) .. +31 of each finished block.  The half solved first
// (the top one for L, the bottom one for U) is solved by its first wavefront;
// the other half's wavefronts subtract its contribution through the
// off-diagonal 64x64 tile (in registers since the start), and that half's
// first wavefront solves it and raises the block's flag.
template <typename T, bool LOWER>
__global__ __launch_bounds__(512) void k_trsv128(int64_t n, const T* __restrict__ A, int64_t lda, T* __restrict__ x,
                                                 uint32_t* __restrict__ flags, uint64_t* __restrict__ ticket,
                                                 uint64_t tbase, uint32_t epoch, int32_t* __restrict__ err) {
  __shared__ T s_part[8][64];
  __shared__ T s_diag[2][64 * 64];
  __shared__ T s_x[64];
  __shared__ int64_t s_blk;
  __shared__ int s_ready;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rh = wave >> 2, cw = wave & 3;
  const int fh = LOWER ? 0 : 1, sh = 1 - fh;
  const int64_t nblk = (n + TB2 - 1) / TB2;
  if (tid == 0) s_blk = (int64_t)(atomicAdd((unsigned long long*)ticket, 1ull) - tbase);
  __syncthreads();
  const int64_t q = s_blk;
  if (q < 0 || q >= nblk) {  // ticket bookkeeping out of step: report, touch nothing
    if (tid == 0) *err = 2;
    return;
  }
  const int64_t b = LOWER ? q : (nblk - 1 - q);
  const int64_t r0 = b * TB2;
  const int64_t row = r0 + rh * 64 + lane;
  const bool rok = row < n;
  T acc = T(0);
  const int64_t ndep = LOWER ? b : (nblk - 1 - b);
  // both diagonal blocks staged in LDS before the waits, column-major
  for (int e = tid; e < 2 * 64 * 64; e += 512) {
    const int h = e >> 12, c = (e >> 6) & 63, rr = e & 63;
    const int64_t gr = r0 + h * 64 + rr, gc = r0 + h * 64 + c;
    s_diag[h][c * 64 + rr] = (gr < n && gc < n) ? A[gr + gc * lda] : T(0);
  }
  T ofd[16];  // off-diagonal tile: second half's rows, first half's columns
  {
    const int64_t c0 = r0 + fh * 64 + cw * 16;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int64_t c = c0 + cc;
      ofd[cc] = (rh == sh && c < n && rok) ? A[row + c * lda] : T(0);
    }
  }
  T apf[32];  // adjacent finished block, loaded before its flag
  const int64_t lastd = ndep - 1;
  if (ndep > 0) {
    const int64_t c0 = (LOWER ? lastd : (nblk - 1 - lastd)) * TB2 + cw * 32;
#pragma unroll
    for (int cc = 0; cc < 32; ++cc) {
      const int64_t c = c0 + cc;
      apf[cc] = (c < n && rok) ? A[row + c * lda] : T(0);
    }
  }
  int64_t done = 0;
  long spins = 0;
  while (done < ndep) {
    if (wave == 0) {
      const int64_t d0 = done + lane;
      const int64_t blk = LOWER ? d0 : (nblk - 1 - d0);
      bool ok = true;
      if (d0 < ndep) ok = __hip_atomic_load(&flags[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      const unsigned long long notready = __ballot(!ok);
      const int nready = notready ? (__ffsll((long long)notready) - 1) : 64;
      if (lane == 0) s_ready = nready;
    }
    __syncthreads();
    int nready = s_ready;
    if (nready == 0) {
      if (++spins > (1L << 22)) {
        if (tid == 0) *err = 1;
        nready = (int)(ndep - done);  // give up waiting (results invalid, flagged)
      } else {
        __syncthreads();
        continue;
      }
    }
    for (int64_t d = done; d < done + nready && d < lastd; ++d) {
      const int64_t blk = LOWER ? d : (nblk - 1 - d);
      const int64_t c0 = blk * TB2 + cw * 32;
      // two rounds of 16 columns, all loads of a round in flight together
#pragma unroll 1
      for (int hh = 0; hh < 32; hh += 16) {
        T av[16], xw[16];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
          const int64_t c = c0 + hh + cc;
          av[cc] = (c < n && rok) ? A[row + c * lda] : T(0);
          xw[cc] = (c < n) ? ld_coh(&x[c]) : T(0);
        }
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) acc = acc - av[cc] * xw[cc];
      }
    }
    done += nready;
    __syncthreads();
  }
  if (ndep > 0) {
    const int64_t c0 = (LOWER ? lastd : (nblk - 1 - lastd)) * TB2 + cw * 32;
    T xv[32];
#pragma unroll
    for (int cc = 0; cc < 32; ++cc) xv[cc] = (c0 + cc < n) ? ld_coh(&x[c0 + cc]) : T(0);
#pragma unroll
    for (int cc = 0; cc < 32; ++cc) acc = acc - apf[cc] * xv[cc];
  }
  s_part[wave][lane] = acc;
  __syncthreads();
  if (wave == fh * 4) {
    T v = rok ? x[row] : T(0);
    v = v + s_part[fh * 4 + 0][lane] + s_part[fh * 4 + 1][lane] + s_part[fh * 4 + 2][lane] + s_part[fh * 4 + 3][lane];
    v = solve64<T, LOWER>(v, s_diag[fh], lane, rok);
    s_x[lane] = v;
    if (rok) st_coh(&x[row], v);
    // stores complete before the barrier, so before the flag raised after it
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  __syncthreads();
  if (rh == sh) {
    T t = acc;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) t = t - ofd[cc] * s_x[cw * 16 + cc];
    s_part[wave][lane] = t;
  }
  __syncthreads();
  if (wave == sh * 4) {
    T v = rok ? x[row] : T(0);
    v = v + s_part[sh * 4 + 0][lane] + s_part[sh * 4 + 1][lane] + s_part[sh * 4 + 2][lane] + s_part[sh * 4 + 3][lane];
    v = solve64<T, LOWER>(v, s_diag[sh], lane, rok);
    if (rok) st_coh(&x[row], v);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (lane == 0) __hip_atomic_store(&flags[b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// partial[c][i] = sum over the c-th chunk of columns of A(i, j) * x(j)
__global__ __launch_bounds__(256) void k_gemv_part(int64_t n, const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ x, int64_t chunk,
                                                   double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t j0 = c * chunk, j1 = (j0 + chunk < n) ? j0 + chunk : n;
  if (i >= n) return;
  double s0 = 0.0, s1 = 0.0;
  int64_t j = j0;
  for (; j + 1 < j1; j += 2) {
    s0 = fma(A[i + j * lda], x[j], s0);
    s1 = fma(A[i + (j + 1) * lda], x[j + 1], s1);
  }
  if (j < j1) s0 = fma(A[i + j * lda], x[j], s0);
  part[c * n + i] = s0 + s1;
}

// r = b - sum_c partial[c] (fixed order)
__global__ void k_gemv_fin(int64_t n, int64_t nchunk, const double* __restrict__ part, const double* __restrict__ b,
                           double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += part[c * n + i];
  r[i] = b[i] - s;
}

// out[0] = max |v| (bit pattern of a non-negative double orders like the value)
__global__ void k_absmax(int64_t n, const double* __restrict__ v, unsigned long long* __restrict__ out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    m = fmax(m, fabs(v[i]));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(s[0]));
}

// row absolute sums of A (FP64): part[c][i] over column chunks
__global__ __launch_bounds__(256) void k_rowabs_part(int64_t n, const double* __restrict__ A, int64_t lda,
                                                     int64_t chunk, double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t j0 = c * chunk, j1 = (j0 + chunk < n) ? j0 + chunk : n;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) s += fabs(A[i + j * lda]);
  part[c * n + i] = s;
}

__global__ void k_rowabs_fin(int64_t n, int64_t nchunk, const double* __restrict__ part,
                             unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (i < n)
    for (int64_t c = 0; c < nchunk; ++c) s += part[c * n + i];
  __shared__ double sm[256];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sm[0]));
}

__global__ void k_d2s_mat(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                          float* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  for (int64_t jj = j; jj < cols; jj += gridDim.y)
    if (i < rows) dst[i + jj * ldd] = (float)src[i + jj * lds];
}

__global__ void k_d2s_vec(int64_t n, const double* __restrict__ s, float* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

// y = x + alpha * (double)z  (alpha applied in FP64)
__global__ void k_axpy_s2d(int64_t n, double alpha, const float* __restrict__ z, const double* __restrict__ x,
                           double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i] + alpha * (double)z[i];
}

__global__ void k_s2d_scaled(int64_t n, double alpha, const float* __restrict__ z, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = alpha * (double)z[i];
}

// partial dot products of w with the columns 0..k-1 of V: part[blk][c]
__global__ __launch_bounds__(256) void k_mdot_part(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double s[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double wi = i < n ? w[i] : 0.0;
  for (int c = 0; c < k; ++c) {
    s[threadIdx.x] = (i < n) ? V[i + c * ldv] * wi : 0.0;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * k + c] = s[0];
    __syncthreads();
  }
}

__global__ void k_mdot_fin(int64_t nb, int k, const double* __restrict__ part, double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s += part[b * k + c];
  out[c] = s;
}

// w -= V(:, 0:k) * h   (h on the device)
__global__ void k_mgemv_sub(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                            const double* __restrict__ h, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int c = 0; c < k; ++c) s -= V[i + c * ldv] * h[c];
  w[i] = s;
}

// y += V(:, 0:k) * c   (c on the device)
__global__ void k_mgemv_add(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                            const double* __restrict__ c, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = y[i];
  for (int q = 0; q < k; ++q) s += V[i + q * ldv] * c[q];
  y[i] = s;
}

__global__ void k_scale_copy(int64_t n, double alpha, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = alpha * src[i];
}

__global__ void k_add(int64_t n, const double* __restrict__ d, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] += d[i];
}

// dst[i] = (float)(src[perm[i]] / s) with s = *smax (a non-negative double's
// bit pattern): the row permutation of the factorization and a scaling that
// keeps the FP32 right-hand side away from under- and overflow.  A zero or
// non-finite s leaves the values unscaled.
__global__ void k_gather_scale(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ src,
                               const unsigned long long* __restrict__ smax, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double sv = __longlong_as_double((long long)*smax);
  const double inv = (sv > 0.0 && sv < 1.0e308) ? 1.0 / sv : 1.0;
  dst[i] = (float)(src[perm[i]] * inv);
}

// y[i] = x[i] + sign * s * (double)z[i] with s = *smax as above (y may be x)
__global__ void k_axpy_dev(int64_t n, double sign, const unsigned long long* __restrict__ smax,
                           const float* __restrict__ z, const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double sv = __longlong_as_double((long long)*smax);
  const double sc = (sv > 0.0 && sv < 1.0e308) ? sv : 1.0;
  const double xi = x ? x[i] : 0.0;
  y[i] = xi + sign * sc * (double)z[i];
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
__global__ void k_diag_zero(int64_t n, const T* __restrict__ A, int64_t lda, int32_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n && A[k + k * lda] == T(0)) *flag = 1;
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t trsv_wave(hipStream_t s, bool lower, int64_t n, const T* A, int64_t lda, T* x, TrsvState* st) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = (n + TB - 1) / TB;
  if (nblk > st->max_blocks) return hipErrorInvalidValue;
  if (st->epoch > 0xF0000000u) return hipErrorInvalidValue;  // caller resets
  st->epoch += 1;
  const uint64_t tbase = st->tickets;
  hipError_t e;
  if (n >= kTrsvWideMinN) {
    const int64_t nblk2 = (n + TB2 - 1) / TB2;
    st->tickets += (uint64_t)nblk2;
    if (lower)
      hipLaunchKernelGGL((k_trsv128<T, true>), dim3((unsigned)nblk2), dim3(512), 0, s, n, A, lda, x, st->flags,
                         st->ticket, tbase, st->epoch, st->err);
    else
      hipLaunchKernelGGL((k_trsv128<T, false>), dim3((unsigned)nblk2), dim3(512), 0, s, n, A, lda, x, st->flags,
                         st->ticket, tbase, st->epoch, st->err);
    e = hipGetLastError();
  } else {
    st->tickets += (uint64_t)nblk;
    if (lower)
      hipLaunchKernelGGL((k_trsv<T, true>), dim3((unsigned)nblk), dim3(256), 0, s, n, A, lda, x, st->flags,
                         st->ticket, tbase, st->epoch, st->err);
    else
      hipLaunchKernelGGL((k_trsv<T, false>), dim3((unsigned)nblk), dim3(256), 0, s, n, A, lda, x, st->flags,
                         st->ticket, tbase, st->epoch, st->err);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {  // nothing ran: the host's counts go back to the device's
    st->tickets = tbase;
    st->epoch -= 1;
  }
  return e;
}
template <typename T>
hipError_t diag_zero_check(hipStream_t s, int64_t n, const T* A, int64_t lda, int32_t* flag) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_zero<T>, dim3(grid1(n)), dim3(256), 0, s, n, A, lda, flag);
  return hipGetLastError();
}
template hipError_t diag_zero_check<double>(hipStream_t, int64_t, const double*, int64_t, int32_t*);
template hipError_t diag_zero_check<float>(hipStream_t, int64_t, const float*, int64_t, int32_t*);

template hipError_t trsv_wave<double>(hipStream_t, bool, int64_t, const double*, int64_t, double*, TrsvState*);
template hipError_t trsv_wave<float>(hipStream_t, bool, int64_t, const float*, int64_t, float*, TrsvState*);

hipError_t residual(hipStream_t s, int64_t n, const double* A, int64_t lda, const double* x, const double* b,
                    double* r, double* part, int64_t nchunk) {
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_gemv_part, dim3(grid1(n), (unsigned)nchunk), dim3(256), 0, s, n, A, lda, x, chunk, part);
  hipLaunchKernelGGL(k_gemv_fin, dim3(grid1(n)), dim3(256), 0, s, n, nchunk, part, b, r);
  return hipGetLastError();
}

hipError_t absmax(hipStream_t s, int64_t n, const double* v, unsigned long long* out) {
  unsigned g = grid1(n);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_absmax, dim3(g), dim3(256), 0, s, n, v, out);
  return hipGetLastError();
}

hipError_t norm_inf_mat(hipStream_t s, int64_t n, const double* A, int64_t lda, double* part, int64_t nchunk,
                        unsigned long long* out) {
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_rowabs_part, dim3(grid1(n), (unsigned)nchunk), dim3(256), 0, s, n, A, lda, chunk, part);
  hipLaunchKernelGGL(k_rowabs_fin, dim3(grid1(n)), dim3(256), 0, s, n, nchunk, part, out);
  return hipGetLastError();
}

hipError_t d2s_mat(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst,
                   int64_t ldd) {
  const unsigned gy = (unsigned)(cols < 65535 ? cols : 65535);
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2s_mat, dim3(grid1(rows), gy), dim3(256), 0, s, rows, cols, src, lds, dst, ldd);
  return hipGetLastError();
}

hipError_t d2s_vec(hipStream_t s, int64_t n, const double* src, float* dst) {
  hipLaunchKernelGGL(k_d2s_vec, dim3(grid1(n)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t axpy_s2d(hipStream_t s, int64_t n, double alpha, const float* z, const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy_s2d, dim3(grid1(n)), dim3(256), 0, s, n, alpha, z, x, y);
  return hipGetLastError();
}

hipError_t s2d_scaled(hipStream_t s, int64_t n, double alpha, const float* z, double* y) {
  hipLaunchKernelGGL(k_s2d_scaled, dim3(grid1(n)), dim3(256), 0, s, n, alpha, z, y);
  return hipGetLastError();
}

hipError_t mdot(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* part,
                double* out) {
  const unsigned nb = grid1(n);
  hipLaunchKernelGGL(k_mdot_part, dim3(nb), dim3(256), 0, s, n, k, V, ldv, w, part);
  hipLaunchKernelGGL(k_mdot_fin, dim3(1), dim3(64), 0, s, (int64_t)nb, k, part, out);
  return hipGetLastError();
}

hipError_t mgemv_sub(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w) {
  hipLaunchKernelGGL(k_mgemv_sub, dim3(grid1(n)), dim3(256), 0, s, n, k, V, ldv, h, w);
  return hipGetLastError();
}

hipError_t mgemv_add(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* c, double* y) {
  hipLaunchKernelGGL(k_mgemv_add, dim3(grid1(n)), dim3(256), 0, s, n, k, V, ldv, c, y);
  return hipGetLastError();
}

hipError_t scale_copy(hipStream_t s, int64_t n, double alpha, const double* src, double* dst) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid1(n)), dim3(256), 0, s, n, alpha, src, dst);
  return hipGetLastError();
}

hipError_t gather_scale(hipStream_t s, int64_t n, const int32_t* perm, const double* src,
                        const unsigned long long* smax, float* dst) {
  hipLaunchKernelGGL(k_gather_scale, dim3(grid1(n)), dim3(256), 0, s, n, perm, src, smax, dst);
  return hipGetLastError();
}

hipError_t axpy_dev(hipStream_t s, int64_t n, double sign, const unsigned long long* smax, const float* z,
                    const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(grid1(n)), dim3(256), 0, s, n, sign, smax, z, x, y);
  return hipGetLastError();
}

hipError_t vec_add(hipStream_t s, int64_t n, const double* d, double* x) {
  hipLaunchKernelGGL(k_add, dim3(grid1(n)), dim3(256), 0, s, n, d, x);
  return hipGetLastError();
}

}  // namespace lupp
