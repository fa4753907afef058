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
// Steps 2-5 update only the rest of a 128-column outer block; the columns
// right of it get one update per outer block with its 128 reflectors
// (k_qr_larft_big builds that T; T^T W and V W both run on the GEMM, K = 128),
// so the trailing matrix is read and written once per 128 columns.
#include "handle.h"
#include "wave.h"

namespace lupp {

namespace {

constexpr int kQrW = 32;         // block width (columns per panel launch)
constexpr int kQrNB = 128;       // outer block width (columns per trailing update)
constexpr int64_t kQrOverlapMin = (int64_t)1 << 26;  // rows x columns of a rest update worth overlapping
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
        // Records in chunks of RC: a chunk's loads are issued together, then
        // tag-checked (a check inside each load's block would make every load
        // wait for the one before), then its exchanges, then the sum in record
        // order.  A chunk wholly past the last workgroup is skipped.
        constexpr int RC = 8, RPW = kQrMaxGroups / NW;
        static_assert(RPW % RC == 0, "record chunks");
        double acc = 0.0;
        long spins = 0;
#pragma unroll
        for (int t0 = 0; t0 < RPW; t0 += RC) {
          if (wave + NW * t0 < G) {  // uniform in the wavefront
            uint64_t u[RC];
#pragma unroll
            for (int t = 0; t < RC; ++t) u[t] = 0;
            for (;;) {
#pragma unroll
              for (int t = 0; t < RC; ++t) {
                const int q = wave + NW * (t0 + t);
                if (q < G) u[t] = qld(&ws->rec[par][q][lane]);
              }
              bool ok = true;
#pragma unroll
              for (int t = 0; t < RC; ++t) {
                const int q = wave + NW * (t0 + t);
                if (q < G) ok &= (uint32_t)(u[t] >> 32) == tag;
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
            uint32_t lo[RC];
#pragma unroll
            for (int t = 0; t < RC; ++t) {
              const int q = wave + NW * (t0 + t);
              lo[t] = 0;
              if (q < G) lo[t] = (uint32_t)__shfl_down((int)(uint32_t)u[t], 1, 64);
            }
#pragma unroll
            for (int t = 0; t < RC; ++t) {
              const int q = wave + NW * (t0 + t);
              if (q < G) acc += __longlong_as_double((long long)(((uint64_t)(uint32_t)u[t] << 32) | lo[t]));
            }
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

// Partials of W = V^T X over row chunks: V is r x LDW (ldv), X is r x N
// (ldx); workgroup (tile, chunk) computes all LDW rows of W for 64 columns
// (X is read once) and writes part[chunk] (column-major LDW x N per chunk).
// Four wavefronts: for LDW = 128 each takes 32 rows x 64 columns (8 MFMA
// accumulators of 16x16), for LDW = 32 each 16 rows x 32 columns (2).  LDS
// tiles of 16 rows, double-buffered: the next tile's loads are in flight
// while the current one is multiplied (50 KB of LDS for LDW = 128, so that
// three workgroups share a CU).
constexpr int kTnCols = 64;
constexpr int kTnTarget = 768;  // workgroups of one product (three per CU)
template <int LDW>
constexpr int tn_k() {
  return LDW >= 64 ? 16 : 32;  // rows per LDS tile
}
template <int LDW>
__global__ __launch_bounds__(256) void k_qr_tn(int64_t r, int64_t N, const double* __restrict__ V, int64_t ldv,
                                               const double* __restrict__ X, int64_t ldx, int64_t rows_per_chunk,
                                               double* __restrict__ part) {
  typedef Mfma<double> MF;
  constexpr int WR = LDW >= 64 ? LDW / 4 : 16;  // rows of W per wavefront
  constexpr int WC = LDW >= 64 ? 64 : 32;       // columns per wavefront
  constexpr int FI = WR / 16, FJ = WC / 16;
  constexpr int kTnK = tn_k<LDW>();
  constexpr int EV = kTnK * LDW / 256, EX = kTnK * kTnCols / 256;
  __shared__ double sV[2][kTnK][LDW + 1];
  __shared__ double sX[2][kTnK][kTnCols + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kTnCols;
  const int64_t chunk = blockIdx.y;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < r) ? r0 + rows_per_chunk : r;
  const int wi = LDW >= 64 ? WR * wave : (wave & 1) * 16;
  const int wc = LDW >= 64 ? 0 : (wave >> 1) * 32;
  MF::v4 acc[FI][FJ];
#pragma unroll
  for (int a = 0; a < FI; ++a)
#pragma unroll
    for (int t = 0; t < FJ; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[a][t][q] = 0.0;
  double rv[EV], rx[EX];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < EV; ++u) {
      const int e = tid + 256 * u, kk = e % kTnK, c = e / kTnK;
      const int64_t row = k0 + kk;
      rv[u] = row < r1 ? V[row + (int64_t)c * ldv] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EX; ++u) {
      const int e = tid + 256 * u, kk = e % kTnK, c = e / kTnK;
      const int64_t row = k0 + kk, col = c0 + c;
      rx[u] = (row < r1 && col < N) ? X[row + col * ldx] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < EV; ++u) {
      const int e = tid + 256 * u;
      sV[buf][e % kTnK][e / kTnK] = rv[u];
    }
#pragma unroll
    for (int u = 0; u < EX; ++u) {
      const int e = tid + 256 * u;
      sX[buf][e % kTnK][e / kTnK] = rx[u];
    }
  };
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t nsteps = (r1 - r0 + kTnK - 1) / kTnK;
  if (nsteps > 0) {
    gload(r0);
    sstore(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < nsteps) gload(r0 + (st + 1) * kTnK);
#pragma unroll
    for (int kk = 0; kk < kTnK; kk += 4) {
      double va[FI], xb[FJ];
#pragma unroll
      for (int a = 0; a < FI; ++a) va[a] = sV[buf][kk + lk][wi + 16 * a + lr];  // A = V^T: A[i][k] = V[k][i]
#pragma unroll
      for (int t = 0; t < FJ; ++t) xb[t] = sX[buf][kk + lk][wc + 16 * t + lr];  // B[k][c] = X[k][c]
#pragma unroll
      for (int a = 0; a < FI; ++a)
#pragma unroll
        for (int t = 0; t < FJ; ++t) acc[a][t] = MF::mma(va[a], xb[t], acc[a][t]);
    }
    if (st + 1 < nsteps) sstore(buf ^ 1);
    __syncthreads();
  }
  // lane holds D[4q + (lane >> 4)][lane & 15] of each 16x16 product
  double* out = part + chunk * (int64_t)LDW * N;
#pragma unroll
  for (int a = 0; a < FI; ++a)
#pragma unroll
    for (int t = 0; t < FJ; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = wi + 16 * a + 4 * q + (lane >> 4);
        const int64_t col = c0 + wc + 16 * t + (lane & 15);
        if (col < N) out[row + col * LDW] = acc[a][t][q];
      }
}

// W = sum of the chunk partials, in chunk order (ldw x N, column-major).
__global__ void k_qr_reduce(int64_t N, int ldw, int nchunk, const double* __restrict__ part, double* __restrict__ Wm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ldw * N) return;
  double t = 0.0;
  for (int c = 0; c < nchunk; ++c) t += part[(int64_t)c * ldw * N + e];
  Wm[e] = t;
}

// t + sum_{l = lo}^{hi - 1} a[l * sa] * g[l] in increasing l (LDS operands):
// eight pairs are loaded before their eight FMAs, so the chain waits for LDS
// once per eight terms rather than once per term; the order of the sum is
// that of the plain loop.
__device__ __forceinline__ double ordered_dot(const double* a, int sa, const double* g, int lo, int hi) {
  double t = 0.0;
  int l = lo;
  for (; l + 8 <= hi; l += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] = a[(l + u) * sa];
      y[u] = g[l + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) t += x[u] * y[u];
  }
  for (; l < hi; ++l) t += a[l * sa] * g[l];
  return t;
}

// One level of block merges in k_qr_larft_big: the 128 / (2 W) pairs of
// W-column blocks, 64 rows in all, four threads per row, each with W / 4
// columns in registers.  Sums run in increasing l (one G load per term of a
// row, feeding W / 4 columns; the next load is in flight during the FMAs).
template <int W>
__device__ __forceinline__ void larft_merge(double (*sT)[kQrNB + 1], const double* __restrict__ Gm, int tid) {
  constexpr int CR = W / 4;
  const int R = tid >> 2, cq = tid & 3;
  const int pr = R / W, ii = R % W, o = 2 * W * pr, c0 = cq * CR;
  double acc[CR];
#pragma unroll
  for (int u = 0; u < CR; ++u) acc[u] = 0.0;
  // X[ii][c] = sum_{l <= c} G[o + ii][o + W + l] T2[l][c]
  const int lend = c0 + CR;  // l <= c < c0 + CR
  double g = Gm[(o + ii) + (o + W) * kQrNB];
  for (int l = 0; l < lend; ++l) {
    const double gn = (l + 1 < lend) ? Gm[(o + ii) + (o + W + l + 1) * kQrNB] : 0.0;
    // every column's value read, the terms with l > c selected away (adding
    // +0.0 leaves a sum that started at +0.0 unchanged; a guarded read per
    // column would wait for the one before it)
    double tv[CR];
#pragma unroll
    for (int u = 0; u < CR; ++u) tv[u] = sT[o + W + l][o + W + c0 + u];
#pragma unroll
    for (int u = 0; u < CR; ++u) acc[u] += (l <= c0 + u) ? g * tv[u] : 0.0;
    g = gn;
  }
#pragma unroll
  for (int u = 0; u < CR; ++u) sT[o + W + c0 + u][o + ii] = acc[u];
  __syncthreads();
  // T12[ii][c] = -sum_{l >= ii} T1[ii][l] X[l][c]
#pragma unroll
  for (int u = 0; u < CR; ++u) acc[u] = 0.0;
  for (int l = ii; l < W; ++l) {
    const double t1 = sT[o + ii][o + l];
#pragma unroll
    for (int u = 0; u < CR; ++u) acc[u] += t1 * sT[o + W + c0 + u][o + l];
  }
#pragma unroll
  for (int u = 0; u < CR; ++u) sT[o + ii][o + W + c0 + u] = -acc[u];
  __syncthreads();
}

// -T^T of the compact WY form of up to 128 reflectors (the 128-column outer
// block), from G = V^T V (128 x 128) and tau (b values), written transposed
// and negated (128 x 128, column-major) for the product W := T^T W =
// 0 - (-T^T) W on the GEMM.  T is built by blocks, with the column recurrence
// T[:j, j] = -tau_j T[:j, :j] G[:j, j] only inside 32-column blocks: for
// V = [V1 V2], Q = (I - V1 T1 V1^T)(I - V2 T2 V2^T) = I - V T V^T with
// T = [T1, -T1 G12 T2; 0, T2], G12 = V1^T V2.  The four 32-column blocks run
// at once (one wavefront each), then two 32 + 32 merges, then one 64 + 64
// merge.  G's pieces are staged in T's strictly lower triangle, which T does
// not use.
__global__ __launch_bounds__(256) void k_qr_larft_big(int b, const double* __restrict__ Gm,
                                                      const double* __restrict__ tau, double* __restrict__ Tneg) {
  __shared__ double sT[kQrNB][kQrNB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kQrNB * (kQrNB + 1); e += 256) (&sT[0][0])[e] = 0.0;
  __syncthreads();
  // 32-column diagonal blocks: G[c0 + l][c0 + j] (l < j) staged at
  // sT[c0 + j][c0 + l]; lane i < j forms T[c0 + i][c0 + j] from its own row
  {
    const int c0 = 32 * wave;
    for (int e = lane; e < 32 * 32; e += 64) {
      const int l = e % 32, jj = e / 32;
      if (l < jj) sT[c0 + jj][c0 + l] = Gm[(c0 + l) + (c0 + jj) * kQrNB];
    }
    __syncthreads();
    for (int jj = 0; jj < 32 && c0 + jj < b; ++jj) {
      const double tj = tau[c0 + jj];
      if (lane < jj) sT[c0 + lane][c0 + jj] = -tj * ordered_dot(&sT[c0 + lane][c0], 1, &sT[c0 + jj][c0], lane, jj);
      if (lane == jj) sT[c0 + jj][c0 + jj] = tj;
    }
  }
  __syncthreads();
  // merges of width 32, then 64: block pairs at o = 2 W p.  X = G12 T2 goes
  // to the strictly lower block sT[o + W + c][o + i] (transposed), then
  // T12 = -T1 X to sT[o + i][o + W + c]
  larft_merge<32>(sT, Gm, tid);
  larft_merge<64>(sT, Gm, tid);
  // Tneg[i][l] = -T[l][i] (T upper triangular; the lower triangle holds G)
  for (int e = tid; e < kQrNB * kQrNB; e += 256) {
    const int i = e % kQrNB, l = e / kQrNB;
    Tneg[e] = (l <= i) ? -sT[l][i] : 0.0;
  }
}

__global__ void k_qr_zero(int64_t count, double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

// T of the compact WY form from G = V^T V (32 x 32) and tau (b values, the
// rest 0): one wavefront; column j after column j-1.  G is staged in LDS
// first.
__global__ __launch_bounds__(64) void k_qr_larft(int b, const double* __restrict__ Gm, const double* __restrict__ tau,
                                                 double* __restrict__ Tm) {
  __shared__ double sT[kQrW][kQrW];
  __shared__ double sG[kQrW * kQrW];
  const int lane = threadIdx.x;
  for (int e = lane; e < kQrW * kQrW; e += 64) {
    sT[e % kQrW][e / kQrW] = 0.0;
    sG[e] = Gm[e];
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    const double tj = tau[j];
    double t = 0.0;
    // (T[:j, :j] G[:j, j])[lane], T upper triangular
    if (lane < j) t = -tj * ordered_dot(&sT[lane][0], 1, sG + j * kQrW, lane, j);
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
  int64_t ch = (kTnTarget + tiles - 1) / tiles;  // about kTnTarget workgroups in all
  const int64_t maxch = (r + 1023) / 1024;  // at least 1024 rows per chunk
  if (ch > maxch) ch = maxch;
  return ch < 1 ? 1 : ch;
}

}  // namespace

// out (ldw x N) = V^T X for V of ldw (32, 64 or 128) columns.  The rows are
// split into chunks as for a product of chunk_width columns (default N), so
// that products over parts of the same columns add their row chunks in the
// same order.
hipError_t qr_tn(hipStream_t s, int64_t r, int64_t N, const double* V, int64_t ldv, const double* X, int64_t ldx,
                 int ldw, double* part, double* out, int64_t chunk_width) {
  const int64_t ch = tn_chunks(r, chunk_width > N ? chunk_width : N);
  int64_t rpc = (r + ch - 1) / ch;
  rpc = (rpc + 31) / 32 * 32;  // a multiple of every tile depth
  const int64_t nch = (r + rpc - 1) / rpc;
  const dim3 grid((unsigned)((N + kTnCols - 1) / kTnCols), (unsigned)nch);
  if (ldw == kQrNB)
    hipLaunchKernelGGL(k_qr_tn<kQrNB>, grid, dim3(256), 0, s, r, N, V, ldv, X, ldx, rpc, part);
  else if (ldw == 64)
    hipLaunchKernelGGL(k_qr_tn<64>, grid, dim3(256), 0, s, r, N, V, ldv, X, ldx, rpc, part);
  else
    hipLaunchKernelGGL(k_qr_tn<kQrW>, grid, dim3(256), 0, s, r, N, V, ldv, X, ldx, rpc, part);
  const int64_t tot = (int64_t)ldw * N;
  hipLaunchKernelGGL(k_qr_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, ldw, (int)nch, part, out);
  return hipGetLastError();
}

namespace {

}  // namespace

void free_qr(lupp_handle_t h) {
  if (!h->qr) return;
  if (h->qr->slots) (void)hipFree(h->qr->slots);
  if (h->qr->buf) (void)hipFree(h->qr->buf);
  if (h->qr->la) (void)hipFree(h->qr->la);
  for (int e = 0; e < 4; ++e)
    if (h->qr->ev[e]) (void)hipEventDestroy(h->qr->ev[e]);
  delete h->qr;
  h->qr = nullptr;
}

// Vbig (m x 128), G and -T^T (128 x 128 each), G32 and T32, W and W2
// (128 x n each), the chunk partials (at most kTnTarget / tiles + 1 chunks
// of ldw x N with tiles = N / 64, so at most 128 x (64 kTnTarget + n) values).
size_t qr_workspace_bytes(int64_t m, int64_t n) {
  const int64_t nn = n > kQrNB ? n : kQrNB;
  return sizeof(QrSlots) + sizeof(double) * (size_t)((int64_t)kQrNB * m + 2 * kQrNB * kQrNB + 2 * kQrW * kQrW +
                                                     2 * kQrNB * nn + kQrNB * (kTnCols * kTnTarget + nn) + 256);
}

namespace {

}  // namespace

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
  q->m = m;
  q->n = n;
  return hipSuccess;
}


// Buffers of one outer block's work: its V (r x 128, explicit: unit
// diagonal, zeros above, zero columns beyond B; ld r), G = V^T V and -T^T
// (128 x 128 each); the column blocks' G32, T32, W (32 x up to n) and chunk
// partials; the trailing update's W, W2 (128 x its columns) and partials.
struct QrBufs {
  double *V, *G, *Tn;
  double *G32, *T32, *Wf, *partf;
  double *W, *W2, *part;
};

QrBufs qr_default_bufs(lupp_handle_t h) {
  QrWs* q = h->qr;
  const int64_t m = q->m, n = q->n;
  const int64_t nn = n > kQrNB ? n : kQrNB;
  QrBufs w;
  w.V = q->buf;                          // m x 128
  w.G = w.V + (int64_t)kQrNB * m;        // 128 x 128
  w.Tn = w.G + kQrNB * kQrNB;            // 128 x 128: -T^T
  w.G32 = w.Tn + kQrNB * kQrNB;          // 32 x 32
  w.T32 = w.G32 + kQrW * kQrW;           // 32 x 32
  w.W = w.T32 + kQrW * kQrW;             // 128 x n
  w.W2 = w.W + (int64_t)kQrNB * nn;      // 128 x n
  w.part = w.W2 + (int64_t)kQrNB * nn;
  w.Wf = w.W;
  w.partf = w.part;
  return w;
}

// The column blocks of an outer block: factor its first B <= 128 columns of
// the r x ncols matrix A (32-column panels on stream s) and apply each
// panel's compact WY form to the columns right of it up to column ce.  With
// wy, V is written out explicitly for the outer block's own update.
hipError_t qr_factor(lupp_handle_t h, hipStream_t s, int64_t r, int64_t ce, double* A, int64_t lda, double* tau,
                     int64_t B, bool wy, const QrBufs& w) {
  QrWs* q = h->qr;
  if (wy) {  // the outer block's V, zero above each panel's rows
    const int64_t cnt = r * kQrNB;
    hipLaunchKernelGGL(k_qr_zero, dim3((unsigned)((cnt + 255) / 256 < 4096 ? (cnt + 255) / 256 : 4096)), dim3(256), 0,
                       s, cnt, w.V);
    LUPP_TRY(hipGetLastError());
  }
  for (int64_t p0 = 0; p0 < B; p0 += kQrW) {
    const int b = (int)((B - p0 < kQrW) ? (B - p0) : kQrW);
    const int64_t rp = r - p0;
    const int G = (int)((rp + kQrThreads - 1) / kQrThreads);
    if (G > kQrMaxGroups) return hipErrorInvalidValue;
    if (q->epoch > 0xF0000000u) {
      hipLaunchKernelGGL(k_qr_reset, dim3(1), dim3(256), 0, s, q->slots);
      LUPP_TRY(hipGetLastError());
      q->epoch = 0;
    }
    double* Vp = w.V + p0 + p0 * r;  // this panel's V: rows p0.., columns p0.. of the outer block's V (ld r)
    const int t = timer_begin(h, LUPP_PHASE_PANEL, s);
    hipLaunchKernelGGL(k_qr_panel<kQrThreads>, dim3(G), dim3(kQrThreads), 0, s, rp, b, A + p0 + p0 * lda, lda,
                       tau + p0, Vp, r, q->slots, q->epoch);
    LUPP_TRY(hipGetLastError());
    timer_end(h, t, s, 0.0);
    q->epoch += (uint32_t)b + 1u;
    const int64_t nb2 = ce - p0 - b;
    if (nb2 <= 0) continue;
    double* Ab = A + p0 + (p0 + b) * lda;
    const int tu = timer_begin(h, LUPP_PHASE_PANEL_GEMM, s);
    LUPP_TRY(qr_tn(s, rp, kQrW, Vp, r, Vp, r, kQrW, w.partf, w.G32));
    hipLaunchKernelGGL(k_qr_larft, dim3(1), dim3(64), 0, s, b, w.G32, tau + p0, w.T32);
    LUPP_TRY(qr_tn(s, rp, nb2, Vp, r, Ab, lda, kQrW, w.partf, w.Wf));
    hipLaunchKernelGGL(k_qr_trmm, dim3((unsigned)((nb2 + 255) / 256)), dim3(256), 0, s, nb2, w.T32, w.Wf);
    LUPP_TRY(hipGetLastError());
    LUPP_TRY(gemm_sub<double>(s, rp, nb2, kQrW, Vp, r, w.Wf, kQrW, Ab, lda, nullptr, 2));
    timer_end(h, tu, s, 4.0 * (double)rp * (double)nb2 * (double)b);
  }
  return hipSuccess;
}

// G = V^T V and -T^T of the outer block's B reflectors (stream s; w.part),
// timed as part of the trailing update.
hipError_t qr_make_t(lupp_handle_t h, hipStream_t s, int64_t r, int64_t B, const double* tau, const QrBufs& w) {
  const int tu = timer_begin(h, LUPP_PHASE_UPDATE, s);
  LUPP_TRY(qr_tn(s, r, kQrNB, w.V, r, w.V, r, kQrNB, w.part, w.G));
  hipLaunchKernelGGL(k_qr_larft_big, dim3(1), dim3(256), 0, s, (int)B, w.G, tau, w.Tn);
  LUPP_TRY(hipGetLastError());
  timer_end(h, tu, s, 0.0);
  return hipSuccess;
}

// A2 := Q^T A2 = A2 - V (T^T (V^T A2)) for the N columns of A2 (r rows) on
// stream s; the row chunks of V^T A2 are those of a product of chunk_width
// columns.
hipError_t qr_apply(lupp_handle_t h, hipStream_t s, int64_t r, int64_t N, double* A2, int64_t lda, int64_t B,
                    int64_t chunk_width, const QrBufs& w) {
  if (N <= 0) return hipSuccess;
  const int tu = timer_begin(h, LUPP_PHASE_UPDATE, s);
  LUPP_TRY(qr_tn(s, r, N, w.V, r, A2, lda, kQrNB, w.part, w.W, chunk_width));
  const int64_t cnt = (int64_t)kQrNB * N;
  hipLaunchKernelGGL(k_qr_zero, dim3((unsigned)((cnt + 255) / 256 < 4096 ? (cnt + 255) / 256 : 4096)), dim3(256), 0, s,
                     cnt, w.W2);
  LUPP_TRY(hipGetLastError());
  LUPP_TRY(gemm_sub<double>(s, kQrNB, N, kQrNB, w.Tn, kQrNB, w.W, kQrNB, w.W2, kQrNB, nullptr, 2));  // W2 = T^T W
  LUPP_TRY(gemm_sub<double>(s, r, N, kQrNB, w.V, r, w.W2, kQrNB, A2, lda, nullptr, 0));             // A2 -= V W2
  timer_end(h, tu, s, 4.0 * (double)r * (double)N * (double)B);
  return hipSuccess;
}

// One outer block on the handle's stream: factor the first B <= 128 columns
// of the r x ncols matrix A (32-column blocks with their compact WY updates
// inside the outer block) and apply Q^T to the columns B .. ncols-1 with one
// 128-column compact WY update.  Leaves in the workspace the outer block's V
// (r x 128, explicit: unit diagonal, zeros above, zero columns beyond B) and
// -T^T of its compact WY form (128 x 128) whenever there are trailing columns
// or keep_wy is set.
hipError_t qr_outer(lupp_handle_t h, int64_t r, int64_t ncols, double* A, int64_t lda, double* tau, int64_t B,
                    bool keep_wy) {
  hipStream_t s = h->stream;
  const QrBufs w = qr_default_bufs(h);
  const int64_t n2 = ncols - B;
  const bool wy = n2 > 0 || keep_wy;
  // the outer block's remaining columns (or, for an outer block with no
  // trailing columns, every column right of each panel)
  LUPP_TRY(qr_factor(h, s, r, n2 > 0 ? B : ncols, A, lda, tau, B, wy, w));
  if (!wy) return hipSuccess;
  LUPP_TRY(qr_make_t(h, s, r, B, tau, w));
  return qr_apply(h, s, r, n2, A + B * lda, lda, B, n2, w);
}

namespace {

// Bytes of the lookahead buffers beyond the default layout: the second V, G
// and -T^T; W, W2 and partials for the next block's update (128 columns) and
// for the rest (up to n columns).
size_t qr_la_bytes(int64_t m, int64_t n) {
  const int64_t nn = n > kQrNB ? n : kQrNB;
  const int64_t part = (int64_t)kQrNB * (kTnCols * kTnTarget + nn);
  return sizeof(double) * (size_t)((int64_t)kQrNB * m + 2 * kQrNB * kQrNB + 2 * kQrNB * kQrNB + part +
                                   2 * (int64_t)kQrNB * nn + part + 256);
}

hipError_t ensure_qr_la(lupp_handle_t h, int64_t m, int64_t n) {
  QrWs* q = h->qr;
  for (int e = 0; e < 4; ++e)
    if (!q->ev[e]) LUPP_TRY(hipEventCreateWithFlags(&q->ev[e], hipEventDisableTiming));
  const size_t need = qr_la_bytes(m, n);
  if (need > q->la_bytes) {
    LUPP_TRY(hipStreamSynchronize(h->stream));
    if (q->la) (void)hipFree(q->la);
    q->la = nullptr;
    q->la_bytes = 0;
    void* p = nullptr;
    LUPP_TRY(hipMalloc(&p, need));
    q->la = (double*)p;
    q->la_bytes = need;
  }
  return hipSuccess;
}

// Side and bulk streams for a column block whose first panel has G
// workgroups: the CU partition whose panel CUs hold all of them.
bool qr_pair(lupp_handle_t h, int G, hipStream_t* side, hipStream_t* bulk) {
  if (h->side && h->bulk && G <= h->panel_cus) {
    *side = h->side;
    *bulk = h->bulk;
    return true;
  }
  if (h->side2 && h->bulk2 && G <= h->panel_cus2) {
    *side = h->side2;
    *bulk = h->bulk2;
    return true;
  }
  return false;
}

}  // namespace

// Lookahead: while block j's compact WY form is applied to the columns beyond
// block j + 1 on the bulk CUs, block j + 1 (updated first, on the handle's
// stream) is factored on the panel's CUs.  V, G and -T^T alternate between two
// buffers by block parity; the next block's update, the rest and the column
// blocks each have their own scratch.  Every product splits its rows as the
// whole trailing update would, so the result is the loop's, bit for bit.
hipError_t geqrf_la(lupp_handle_t h, int64_t m, int64_t n, double* A, int64_t lda, double* tau) {
  QrWs* q = h->qr;
  hipStream_t s = h->stream;
  const int64_t k = m < n ? m : n;
  const int64_t J = (k + kQrNB - 1) / kQrNB;
  const int64_t nn = n > kQrNB ? n : kQrNB;
  const int64_t part = (int64_t)kQrNB * (kTnCols * kTnTarget + nn);
  QrBufs w[2];
  w[0] = qr_default_bufs(h);
  w[1] = w[0];
  double* x = q->la;
  w[1].V = x;
  x += (int64_t)kQrNB * m;
  w[1].G = x;
  x += kQrNB * kQrNB;
  w[1].Tn = x;
  x += kQrNB * kQrNB;
  // the next block's update on the handle's stream (both parities)
  double* Wn = x;
  x += kQrNB * kQrNB;
  double* W2n = x;
  x += kQrNB * kQrNB;
  double* partn = x;
  x += part;
  // the rest on the bulk stream
  double* Wr = x;
  x += (int64_t)kQrNB * nn;
  double* W2r = x;
  x += (int64_t)kQrNB * nn;
  double* partr = x;
  hipEvent_t ev_f = q->ev[0], ev_rest = q->ev[3];
  bool rest_pending = false, f_side = false;
  // block 0 on the handle's stream
  {
    const int64_t B = k < kQrNB ? k : kQrNB;
    LUPP_TRY(qr_factor(h, s, m, n - B > 0 ? B : n, A, lda, tau, B, n - B > 0, w[0]));
  }
  for (int64_t j = 0; j < J; ++j) {
    const int64_t j0 = j * kQrNB, r = m - j0, B = (k - j0 < kQrNB) ? (k - j0) : kQrNB;
    const int64_t n2 = n - j0 - B;
    double* Aj = A + j0 + j0 * lda;
    const QrBufs& wj = w[j & 1];
    if (f_side) LUPP_TRY(hipStreamWaitEvent(s, ev_f, 0));
    if (rest_pending) LUPP_TRY(hipStreamWaitEvent(s, ev_rest, 0));
    f_side = rest_pending = false;
    if (n2 <= 0) break;  // the last block, factored with its columns
    LUPP_TRY(qr_make_t(h, s, r, B, tau + j0, QrBufs{wj.V, wj.G, wj.Tn, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                 nullptr, partn}));
    const int64_t jn0 = j0 + kQrNB;
    const int64_t Bn = (j + 1 < J) ? ((k - jn0 < kQrNB) ? (k - jn0) : kQrNB) : 0;
    const int64_t nxt = Bn;  // columns the next block's factorization needs first
    hipStream_t side = nullptr, bulk = nullptr;
    const int Gn = Bn > 0 ? (int)((m - jn0 + kQrThreads - 1) / kQrThreads) : 0;
    // overlap only while the rest of the update outlasts the next block's
    // factorization on the panel's CUs (about 8192 x 8192 and up); smaller
    // steps run in order on all CUs
    const bool overlap = Bn > 0 && n2 - nxt > 0 && r * (n2 - nxt) >= kQrOverlapMin && qr_pair(h, Gn, &side, &bulk);
    QrBufs wn = wj, wr = wj;
    wn.W = Wn;
    wn.W2 = W2n;
    wn.part = partn;
    wr.W = Wr;
    wr.W2 = W2r;
    wr.part = partr;
    double* A2 = Aj + B * lda;
    if (!overlap) {
      LUPP_TRY(qr_apply(h, s, r, n2, A2, lda, B, n2, wr));
    } else {
      LUPP_TRY(hipEventRecord(q->ev[1], s));  // T ready
      LUPP_TRY(qr_apply(h, s, r, nxt, A2, lda, B, n2, wn));
      LUPP_TRY(hipEventRecord(q->ev[2], s));  // next block updated
      LUPP_TRY(hipStreamWaitEvent(bulk, q->ev[1], 0));
      LUPP_TRY(qr_apply(h, bulk, r, n2 - nxt, A2 + nxt * lda, lda, B, n2, wr));
      LUPP_TRY(hipEventRecord(ev_rest, bulk));
      rest_pending = true;
    }
    if (Bn > 0) {
      const int64_t n2n = n - jn0 - Bn;
      double* An = A + jn0 + jn0 * lda;
      hipStream_t fs = s;
      if (overlap) {
        LUPP_TRY(hipStreamWaitEvent(side, q->ev[2], 0));
        fs = side;
      }
      LUPP_TRY(qr_factor(h, fs, m - jn0, n2n > 0 ? Bn : n - jn0, An, lda, tau + jn0, Bn, n2n > 0, w[(j + 1) & 1]));
      if (overlap) {
        LUPP_TRY(hipEventRecord(ev_f, side));
        f_side = true;
      }
    }
  }
  if (f_side) LUPP_TRY(hipStreamWaitEvent(s, ev_f, 0));
  if (rest_pending) LUPP_TRY(hipStreamWaitEvent(s, ev_rest, 0));
  return hipSuccess;
}

// P = A (m x n, in place): R on and above the diagonal, the Householder
// vectors below it, tau[min(m, n)].  Outer blocks of 128 columns: each is
// factored as four 32-column blocks (the panel kernel, and the compact WY
// update of the block's remaining columns), then the trailing columns get one
// 128-column compact WY update: W = V^T A2, W := T^T W, A2 -= V W.  With
// lookahead (the handle's default) the next outer block is factored on the
// panel's CUs while the rest of the update runs on the others.
hipError_t geqrf(lupp_handle_t h, int64_t m, int64_t n, double* A, int64_t lda, double* tau) {
  const int64_t k = m < n ? m : n;
  if (k == 0) return hipSuccess;
  LUPP_TRY(ensure_qr(h, m, n));
  if (h->lookahead >= 1 && k > kQrNB && ensure_workspace(h) == hipSuccess && h->lookahead >= 1 && h->side &&
      h->bulk) {
    LUPP_TRY(ensure_qr_la(h, m, n));
    return geqrf_la(h, m, n, A, lda, tau);
  }
  for (int64_t j0 = 0; j0 < k; j0 += kQrNB) {
    const int64_t B = (k - j0 < kQrNB) ? (k - j0) : kQrNB;
    LUPP_TRY(qr_outer(h, m - j0, n - j0, A + j0 + j0 * lda, lda, tau + j0, B, false));
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
