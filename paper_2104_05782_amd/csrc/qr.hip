// Householder QR factorization, blocked right-looking with the compact WY
// form: the paper's HQR (Section 2.2: R upper triangular, V unit lower
// triangular holding the Householder vectors, and their scalars) with the
// products of reflectors applied as I - V T V^T (Section 2.3), so that the
// bulk of the work is matrix-matrix products.
//
// Per block of b <= 32 columns (rows j0 .. m-1):
//   1. k_qr_panel: the block's reflectors, one column at a time, in one
//      cooperative launch (one row per thread, G workgroups of 512 threads).
//      Column j needs two reductions over the rows below its diagonal, sum
//      x_i^2 and sum x_i a_ic for the block's later columns c; each
//      workgroup reduces its rows (a transpose-reduction inside each
//      wavefront: 31 exchanges of halves instead of 32 separate wavefront
//      sums), publishes its 32 partial sums as tagged 64-bit words, and every
//      workgroup adds all partials in a fixed order (deterministic).  Then
//      beta = -sign(alpha) sqrt(alpha^2 + s), tau = (beta - alpha) / beta,
//      v_i = x_i / (alpha - beta), w_c = a_jc + (sum x_i a_ic) / (alpha -
//      beta), and every row applies a_ic -= tau v_i w_c.  The block also goes
//      out as an explicit V (unit diagonal, zeros above, 32 columns).
//   2. k_qr_tn + k_qr_reduce: G = V^T V and W = V^T A2 (split over row chunks,
//      MFMA v_mfma_f64_16x16x4f64 on LDS tiles, chunk partials added in
//      order).
//   3. k_qr_larft: T (upper triangular, Q_block = H_1 ... H_b = I - V T V^T)
//      from G and tau: T[j][j] = tau_j, T[:j, j] = -tau_j T[:j, :j] G[:j, j].
//   4. k_qr_trmm: W := T^T W.
//   5. A2 -= V W on the FP64 MFMA GEMM of the LU path.
#include "handle.h"
#include "wave.h"

namespace lupp {

namespace {

constexpr int kQrW = 32;         // block width (columns per panel launch)
constexpr int kQrThreads = 512;  // rows per workgroup of the panel kernel
constexpr long kQrSpin = 1L << 22;

__device__ __forceinline__ void qst(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t qld(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)u, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(u >> 32), m, 64);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum of 32 values over the 64 lanes of a wavefront: each exchange step sends
// the half of the values the partner keeps, so after five steps lane l holds
// value l >> 1 summed over 32 lanes, and a last step adds the lane pairs.
// Lanes 2i and 2i+1 return the total of value i.  Fixed order.
__device__ __forceinline__ double wave_sum32(double (&v)[32], int lane) {
  static_for<0, 5>([&](auto si) {
    constexpr int s = decltype(si)::value;
    constexpr int h = 16 >> s, m = 32 >> s;
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double send = up ? v[q] : v[q + h];
      const double keep = up ? v[q + h] : v[q];
      v[q] = keep + shfl_xor_d(send, m);
    }
  });
  return v[0] + shfl_xor_d(v[0], 1);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_qr_panel(int64_t r, int w, double* __restrict__ P, int64_t ld,
                                                 double* __restrict__ tau, double* __restrict__ V, int64_t ldv,
                                                 QrSlots* __restrict__ ws, uint32_t epoch) {
  constexpr int W = kQrW, NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int64_t i = (int64_t)g * NT + tid;  // this thread's row
  const bool rok = i < r;
  __shared__ double s_wp[NW][W];   // wavefront partials
  __shared__ double s_tot[W];      // column totals: [0] sum x^2, [c] sum x a_c
  __shared__ double s_row[W];      // row j
  __shared__ int s_broken;
  if (tid == 0) s_broken = 0;

  double a[W];
#pragma unroll
  for (int c = 0; c < W; ++c) a[c] = (rok && c < w) ? P[i + (int64_t)c * ld] : 0.0;
  __syncthreads();

#pragma clang loop unroll(full)
  for (int j = 0; j < W; ++j) {
    if (j < w) {
      const int par = j & 1;
      const uint32_t tag = epoch + 1u + (uint32_t)j;
      // 1. partial sums of the rows below the diagonal
      const bool below = rok && i > j;
      double v[W];
      const double x = below ? a[j] : 0.0;
      v[0] = x * x;
#pragma unroll
      for (int c = 1; c < W; ++c) v[c] = (c > j) ? x * a[c] : 0.0;
      const double ws32 = wave_sum32(v, lane);
      if ((lane & 1) == 0) s_wp[wave][lane >> 1] = ws32;
      if (i == j) {
#pragma unroll
        for (int c = 0; c < W; ++c) s_row[c] = a[c];
      }
      lds_barrier();
      // 2. this workgroup's partials in wavefront order; published
      if (G == 1) {
        if (tid < W) {
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) t += s_wp[q][tid];
          s_tot[tid] = t;
        }
        lds_barrier();
      } else {
        if (wave == 0) {
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) t += s_wp[q][lane >> 1];
          const uint64_t u = (uint64_t)__double_as_longlong(t);
          const uint32_t pay = (lane & 1) ? (uint32_t)u : (uint32_t)(u >> 32);
          qst(&ws->rec[par][g][lane], ((uint64_t)tag << 32) | pay);
          if (g == 0) {
            const uint64_t ur = (uint64_t)__double_as_longlong(s_row[lane >> 1]);
            const uint32_t pr = (lane & 1) ? (uint32_t)ur : (uint32_t)(ur >> 32);
            qst(&ws->rowj[par][lane], ((uint64_t)tag << 32) | pr);
          }
        }
        lds_barrier();  // s_wp is reused below
        // 3. every wavefront adds the records of workgroups wave, wave + NW, ...
        //    (lane = word); wavefront 0 also reads row j
        // (all of a wavefront's records loaded together, then tag-checked)
        constexpr int RPW = kQrMaxGroups / NW;
        uint64_t u[RPW];
        {
          long spins = 0;
          for (;;) {
            bool ok = true;
#pragma unroll
            for (int t = 0; t < RPW; ++t) {
              const int q = wave + NW * t;
              if (q < G) {
                u[t] = qld(&ws->rec[par][q][lane]);
                ok &= (uint32_t)(u[t] >> 32) == tag;
              }
            }
            if (__all(ok)) break;
            if (++spins > kQrSpin || s_broken) {
              if (lane == 0) {
                __hip_atomic_store(&ws->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_broken = 1;
              }
              break;
            }
          }
        }
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < RPW; ++t) {
          const int q = wave + NW * t;
          if (q < G) {  // uniform in the wavefront
            const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)u[t], 1, 64);
            acc += __longlong_as_double((long long)(((uint64_t)(uint32_t)u[t] << 32) | lo));
          }
        }
        if ((lane & 1) == 0) s_wp[wave][lane >> 1] = acc;
        if (wave == 0 && g != 0) {
          uint64_t u = 0;
          long spins = 0;
          for (;;) {
            u = qld(&ws->rowj[par][lane]);
            if (__all((uint32_t)(u >> 32) == tag)) break;
            if (++spins > kQrSpin || s_broken) {
              if (lane == 0) {
                __hip_atomic_store(&ws->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_broken = 1;
              }
              break;
            }
          }
          const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)u, 1, 64);
          if ((lane & 1) == 0) s_row[lane >> 1] = __longlong_as_double((long long)(((uint64_t)(uint32_t)u << 32) | lo));
        }
        lds_barrier();
        if (tid < W) {
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) t += s_wp[q][tid];
          s_tot[tid] = t;
        }
        lds_barrier();
      }
      // 4. the reflector and its application to this thread's row
      const double alpha = s_row[j], ss = s_tot[0];
      if (ss != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        const double t = (beta - alpha) / beta;
        const double den = alpha - beta;
        double tw[W];
#pragma unroll
        for (int c = 0; c < W; ++c) tw[c] = (c > j) ? t * (s_row[c] + s_tot[c] / den) : 0.0;
        if (below) {
          const double vi = a[j] / den;
          a[j] = vi;
#pragma unroll
          for (int c = 0; c < W; ++c)
            if (c > j) a[c] = fma(-tw[c], vi, a[c]);
        } else if (i == j) {
          a[j] = beta;
#pragma unroll
          for (int c = 0; c < W; ++c)
            if (c > j) a[c] -= tw[c];
        }
        if (g == 0 && tid == 0) tau[j] = t;
      } else if (g == 0 && tid == 0) {
        tau[j] = 0.0;
      }
      lds_barrier();  // s_row / s_tot of this column read by everyone
    }
  }
  if (rok) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
      if (c < w) P[i + (int64_t)c * ld] = a[c];
      V[i + (int64_t)c * ldv] = (c < w && i > c) ? a[c] : ((c < w && i == c) ? 1.0 : 0.0);
    }
  }
}

// Partials of W = V^T X over row chunks: V is r x 32 (ldv), X is r x N (ldx);
// workgroup (tile, chunk) writes part[chunk][32 x 64 tile] (column-major 32 x
// N per chunk).  Four wavefronts, each 16 rows x 32 columns of the tile (two
// 16x16 MFMA accumulators); LDS tiles of 32 rows.
constexpr int kTnCols = 64, kTnK = 32;
__global__ __launch_bounds__(256) void k_qr_tn(int64_t r, int64_t N, const double* __restrict__ V, int64_t ldv,
                                               const double* __restrict__ X, int64_t ldx, int64_t rows_per_chunk,
                                               double* __restrict__ part) {
  typedef Mfma<double> MF;
  __shared__ double sV[kTnK][kQrW + 1];
  __shared__ double sX[kTnK][kTnCols + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kTnCols;
  const int64_t chunk = blockIdx.y;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < r) ? r0 + rows_per_chunk : r;
  const int wi = (wave & 1) * 16, wc = (wave >> 1) * 32;  // this wavefront's rows of W and columns of the tile
  MF::v4 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = 0.0;
  for (int64_t k0 = r0; k0 < r1; k0 += kTnK) {
    // V tile: 32 rows x 32 columns, X tile: 32 rows x 64 columns (row index fastest)
#pragma unroll
    for (int e = tid; e < kTnK * kQrW; e += 256) {
      const int kk = e % kTnK, c = e / kTnK;
      const int64_t row = k0 + kk;
      sV[kk][c] = row < r1 ? V[row + (int64_t)c * ldv] : 0.0;
    }
#pragma unroll
    for (int e = tid; e < kTnK * kTnCols; e += 256) {
      const int kk = e % kTnK, c = e / kTnK;
      const int64_t row = k0 + kk, col = c0 + c;
      sX[kk][c] = (row < r1 && col < N) ? X[row + col * ldx] : 0.0;
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < kTnK; kk += 4) {
      const double va = sV[kk + lk][wi + lr];  // A = V^T: A[i][k] = V[k][i]
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double xb = sX[kk + lk][wc + 16 * t + lr];  // B[k][c] = X[k][c]
        acc[t] = MF::mma(va, xb, acc[t]);
      }
    }
    __syncthreads();
  }
  // lane holds D[4q + (lane >> 4)][lane & 15]: W row wi + 4q + (lane >> 4), column wc + 16t + (lane & 15)
  double* out = part + chunk * (int64_t)kQrW * N;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = wi + 4 * q + (lane >> 4);
      const int64_t col = c0 + wc + 16 * t + (lane & 15);
      if (col < N) out[row + col * kQrW] = acc[t][q];
    }
}

// W = sum of the chunk partials, in chunk order (32 x N, column-major).
__global__ void k_qr_reduce(int64_t N, int nchunk, const double* __restrict__ part, double* __restrict__ Wm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)kQrW * N) return;
  double t = 0.0;
  for (int c = 0; c < nchunk; ++c) t += part[(int64_t)c * kQrW * N + e];
  Wm[e] = t;
}

// T of the compact WY form from G = V^T V (32 x 32) and tau (b values, the
// rest 0): one wavefront; column j after column j-1.
__global__ __launch_bounds__(64) void k_qr_larft(int b, const double* __restrict__ Gm, const double* __restrict__ tau,
                                                 double* __restrict__ Tm) {
  __shared__ double sT[kQrW][kQrW];
  const int lane = threadIdx.x;
  for (int e = lane; e < kQrW * kQrW; e += 64) sT[e % kQrW][e / kQrW] = 0.0;
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    const double tj = tau[j];
    double t = 0.0;
    if (lane < j) {
      // (T[:j, :j] G[:j, j])[lane], T upper triangular
      for (int l = lane; l < j; ++l) t += sT[lane][l] * Gm[l + j * kQrW];
      t = -tj * t;
    }
    __syncthreads();
    if (lane < j) sT[lane][j] = t;
    if (lane == j) sT[j][j] = tj;
    __syncthreads();
  }
  for (int e = lane; e < kQrW * kQrW; e += 64) Tm[e] = sT[e % kQrW][e / kQrW];
}

// W := T^T W, one thread per column of W (32 x N).
__global__ __launch_bounds__(256) void k_qr_trmm(int64_t N, const double* __restrict__ Tm, double* __restrict__ Wm) {
  __shared__ double sT[kQrW * kQrW];
  for (int e = threadIdx.x; e < kQrW * kQrW; e += blockDim.x) sT[e] = Tm[e];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double w[kQrW];
#pragma unroll
  for (int l = 0; l < kQrW; ++l) w[l] = Wm[l + c * kQrW];
#pragma unroll
  for (int i = kQrW - 1; i >= 0; --i) {  // row i of T^T W uses rows l <= i
    double t = 0.0;
#pragma unroll
    for (int l = 0; l <= i; ++l) t += sT[l + i * kQrW] * w[l];
    w[i] = t;
  }
#pragma unroll
  for (int l = 0; l < kQrW; ++l) Wm[l + c * kQrW] = w[l];
}

__global__ void k_qr_reset(QrSlots* ws) {
  uint64_t* p = &ws->rec[0][0][0];
  for (int e = threadIdx.x; e < 2 * kQrMaxGroups * 64; e += blockDim.x) p[e] = 0;
  for (int e = threadIdx.x; e < 2 * 64; e += blockDim.x) (&ws->rowj[0][0])[e] = 0;
}

}  // namespace

namespace {

int64_t tn_chunks(int64_t r, int64_t N) {
  const int64_t tiles = (N + kTnCols - 1) / kTnCols;
  int64_t ch = (512 + tiles - 1) / tiles;  // about 512 workgroups in all
  const int64_t maxch = (r + 1023) / 1024;  // at least 1024 rows per chunk
  if (ch > maxch) ch = maxch;
  return ch < 1 ? 1 : ch;
}

hipError_t tn(hipStream_t s, int64_t r, int64_t N, const double* V, int64_t ldv, const double* X, int64_t ldx,
              double* part, double* out) {
  const int64_t ch = tn_chunks(r, N);
  int64_t rpc = (r + ch - 1) / ch;
  rpc = (rpc + kTnK - 1) / kTnK * kTnK;
  const int64_t nch = (r + rpc - 1) / rpc;
  hipLaunchKernelGGL(k_qr_tn, dim3((unsigned)((N + kTnCols - 1) / kTnCols), (unsigned)nch), dim3(256), 0, s, r, N, V,
                     ldv, X, ldx, rpc, part);
  const int64_t tot = (int64_t)kQrW * N;
  hipLaunchKernelGGL(k_qr_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, (int)nch, part, out);
  return hipGetLastError();
}

}  // namespace

void free_qr(lupp_handle_t h) {
  if (!h->qr) return;
  if (h->qr->slots) (void)hipFree(h->qr->slots);
  if (h->qr->buf) (void)hipFree(h->qr->buf);
  delete h->qr;
  h->qr = nullptr;
}

size_t qr_workspace_bytes(int64_t m, int64_t n) {
  const int64_t chmax = 512;
  return sizeof(QrSlots) + sizeof(double) * (size_t)((int64_t)kQrW * m + 3 * kQrW * kQrW + kQrW * n +
                                                     chmax * kQrW * (n > kQrW ? n : kQrW) + 64);
}

namespace {

hipError_t ensure_qr(lupp_handle_t h, int64_t m, int64_t n) {
  if (!h->qr) {
    h->qr = new (std::nothrow) QrWs();
    if (!h->qr) return hipErrorOutOfMemory;
  }
  QrWs* q = h->qr;
  if (!q->slots) {
    LUPP_TRY(hipMalloc(&q->slots, sizeof(QrSlots)));
    LUPP_TRY(hipMemset(q->slots, 0, sizeof(QrSlots)));
    q->epoch = 0;
  }
  const size_t need = qr_workspace_bytes(m, n) - sizeof(QrSlots);
  if (need > q->bytes) {
    LUPP_TRY(hipStreamSynchronize(h->stream));
    if (q->buf) (void)hipFree(q->buf);
    q->buf = nullptr;
    q->bytes = 0;
    LUPP_TRY(hipMalloc(&q->buf, need));
    q->bytes = need;
  }
  return hipSuccess;
}

}  // namespace

// P = A (m x n, in place): R on and above the diagonal, the Householder
// vectors below it, tau[min(m, n)].
hipError_t geqrf(lupp_handle_t h, int64_t m, int64_t n, double* A, int64_t lda, double* tau) {
  const int64_t k = m < n ? m : n;
  if (k == 0) return hipSuccess;
  LUPP_TRY(ensure_qr(h, m, n));
  QrWs* q = h->qr;
  hipStream_t s = h->stream;
  double* Vb = q->buf;                       // m x 32
  double* Gm = Vb + (int64_t)kQrW * m;       // 32 x 32
  double* Tm = Gm + kQrW * kQrW;             // 32 x 32
  double* Wm = Tm + kQrW * kQrW;             // 32 x n
  double* part = Wm + (int64_t)kQrW * n + kQrW * kQrW;
  for (int64_t j0 = 0; j0 < k; j0 += kQrW) {
    const int b = (int)((k - j0 < kQrW) ? (k - j0) : kQrW);
    const int64_t r = m - j0;
    const int G = (int)((r + kQrThreads - 1) / kQrThreads);
    if (G > kQrMaxGroups) return hipErrorInvalidValue;
    if (q->epoch > 0xF0000000u) {
      hipLaunchKernelGGL(k_qr_reset, dim3(1), dim3(256), 0, s, q->slots);
      LUPP_TRY(hipGetLastError());
      q->epoch = 0;
    }
    const int t = timer_begin(h, LUPP_PHASE_PANEL, s);
    hipLaunchKernelGGL(k_qr_panel<kQrThreads>, dim3(G), dim3(kQrThreads), 0, s, r, b, A + j0 + j0 * lda, lda,
                       tau + j0, Vb, r, q->slots, q->epoch);
    LUPP_TRY(hipGetLastError());
    timer_end(h, t, s, 0.0);
    q->epoch += (uint32_t)b + 1u;
    const int64_t n2 = n - j0 - b;
    if (n2 <= 0) continue;
    double* A2 = A + j0 + (j0 + b) * lda;
    const int tu = timer_begin(h, LUPP_PHASE_UPDATE, s);
    LUPP_TRY(tn(s, r, kQrW, Vb, r, Vb, r, part, Gm));
    hipLaunchKernelGGL(k_qr_larft, dim3(1), dim3(64), 0, s, b, Gm, tau + j0, Tm);
    LUPP_TRY(tn(s, r, n2, Vb, r, A2, lda, part, Wm));
    hipLaunchKernelGGL(k_qr_trmm, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, n2, Tm, Wm);
    LUPP_TRY(hipGetLastError());
    LUPP_TRY(gemm_sub<double>(s, r, n2, kQrW, Vb, r, Wm, kQrW, A2, lda, nullptr, 0));
    timer_end(h, tu, s, 4.0 * (double)r * (double)n2 * (double)b);
  }
  return hipSuccess;
}

}  // namespace lupp

extern "C" int lupp_dgeqrf(lupp_handle_t h, int64_t m, int64_t n, double* dA, int64_t lda, double* dtau) {
  if (!h) return -1;
  if (m < 0 || m >= ((int64_t)1 << 31)) return -2;
  if (n < 0) return -3;
  if (!dA && m > 0 && n > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (!dtau && m > 0 && n > 0) return -6;
  if ((m + lupp::kQrThreads - 1) / lupp::kQrThreads > lupp::kQrMaxGroups) return LUPP_ERR_UNSUPPORTED;
  const hipError_t e = lupp::geqrf(h, m, n, dA, lda, dtau);
  return e == hipErrorOutOfMemory ? LUPP_ERR_ALLOC : lupp::hip_status(e);
}
