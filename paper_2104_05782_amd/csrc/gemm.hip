// Trailing-update GEMM  C -= A * B  on MFMA (FP64: v_mfma_f64_16x16x4f64,
// FP32: v_mfma_f32_16x16x4f32), column-major operands of any shape.
//
// This is the update A22 := A22 - A21 * U12 of the right-looking step, the
// operation the paper identifies as the dominant cost of a blocked
// factorization (Section 4.1: the Level-3 BLAS products; Section 5.4: the
// matrix-matrix products form the dominant cost).  It is also used inside the
// recursive column-block factorization and the recursive triangular solves.
//
// Design (gfx950): a workgroup computes a BM x BN tile of C with
// WGM x WGN wavefronts; K is consumed in steps of BK through double-buffered
// LDS tiles (one barrier per step; the next step's global loads are issued
// before the current step's MFMAs).  Edge tiles clamp their load addresses
// into the matrix and zero the loaded value instead of branching, so every
// load is unconditional.  The accumulators are loaded from C at the start
// (FP32: A negated while it is staged, so the MFMAs accumulate C - A*B;
// FP64: from -C, accumulating A*B - C, stored negated), so the epilogue is a
// plain store (no read-modify-write latency at the end).
// Tiles are mapped XCD-aware: consecutive workgroup ids land on different XCDs
// (round robin), so the id is first split into (xcd, slot) and each XCD walks
// its own contiguous band of tiles in groups of 8 tile-rows, keeping the A
// rows and B columns it needs in its own L2.
#include "common.h"

namespace lupp {

constexpr int kXcds = 8;
constexpr int kGroupM = 8;

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int MINB>
__global__ __launch_bounds__(64 * WGM* WGN, MINB) void k_gemm_sub(int64_t M, int64_t N, int64_t K,
                                                                  const T* __restrict__ A, int64_t lda,
                                                                  const T* __restrict__ B, int64_t ldb,
                                                                  T* __restrict__ C, int64_t ldc, int tiles_m,
                                                                  int tiles_n) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int PAD = 16;  // 16-element k-rows (64 B in FP32) land in distinct bank groups
  constexpr int LDSA = BM + PAD, LDSB = BN + PAD;
  constexpr int EA = BM * BK / NT, EB = BK * BN / NT;
  constexpr int KA = NT / BM;  // k-rows of the A tile loaded per pass
  constexpr int NB_ = NT / BK; // columns of the B tile loaded per pass
  static_assert(EA * NT == BM * BK && EB * NT == BK * BN, "tile/thread mismatch");
  static_assert(KA * BM == NT && NB_ * BK == NT, "thread layout");
  typedef typename Mfma<T>::v4 v4;

  __shared__ T sA[2][BK * LDSA];
  __shared__ T sB[2][BK * LDSB];

  // XCD-aware tile order
  const int total = tiles_m * tiles_n;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int bid = blockIdx.x;
  const int t = (bid % kXcds) * per_xcd + bid / kXcds;
  if (t >= total) return;
  const int group_size = kGroupM * tiles_n;
  const int group = t / group_size;
  const int first_m = group * kGroupM;
  const int gm = min(tiles_m - first_m, kGroupM);
  const int within = t - group * group_size;
  const int tm = first_m + within % gm;
  const int tn = within / gm;

  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  // A tile: thread loads row ai = tid % BM, k-rows ak0 + KA*s
  const int ai = tid % BM, ak0 = tid / BM;
  const bool arow_ok = (m0 + ai) < M;
  const T* pa = A + (arow_ok ? (m0 + ai) : (M - 1));
  // B tile: thread loads k-row bk = tid % BK of columns bn0 + NB_*s
  const int bk = tid % BK, bn0 = tid / BK;
  bool bcol_ok[EB];
  const T* pb[EB];
#pragma unroll
  for (int s = 0; s < EB; ++s) {
    const int64_t gn = n0 + bn0 + NB_ * s;
    bcol_ok[s] = gn < N;
    pb[s] = B + (bcol_ok[s] ? gn : (N - 1)) * ldb;
  }

  T ra[EA], rb[EB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int s = 0; s < EA; ++s) {
      const int64_t gk = k0 + ak0 + KA * s;
      const bool ok = arow_ok && gk < K;
      const T v = pa[(gk < K ? gk : K - 1) * lda];
      ra[s] = ok ? v : T(0);
    }
    const int64_t gk = k0 + bk;
    const bool kok = gk < K;
    const int64_t gkc = kok ? gk : K - 1;
#pragma unroll
    for (int s = 0; s < EB; ++s) {
      const T v = pb[s][gkc];
      rb[s] = (kok && bcol_ok[s]) ? v : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < EA; ++s) sA[buf][(ak0 + KA * s) * LDSA + ai] = -ra[s];
#pragma unroll
    for (int s = 0; s < EB; ++s) sB[buf][bk * LDSB + bn0 + NB_ * s] = rb[s];
  };

  // the accumulators start from C (clamped addresses, zero outside): the
  // epilogue is then a plain store and the loads overlap the first tile
  v4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
    const int64_t rowc = row < M ? row : M - 1;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wn * WTN + j * 16 + Mfma<T>::col(lane, r);
        const int64_t colc = col < N ? col : N - 1;
        const T v = C[rowc + colc * ldc];
        acc[i][j][r] = (row < M && col < N) ? v : T(0);
      }
    }
  }

  const int KT = (int)((K + BK - 1) / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  const int arow = wm * WTM + (lane & 15);
  const int bcol = wn * WTN + (lane & 15);
  for (int kt = 0; kt < KT; ++kt) {
    if (kt + 1 < KT) gload((int64_t)(kt + 1) * BK);
    const T* as = sA[kt & 1] + (lane >> 4) * LDSA + arow;
    const T* bs = sB[kt & 1] + (lane >> 4) * LDSB + bcol;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      T af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = as[kk * 4 * LDSA + i * 16];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = bs[kk * 4 * LDSB + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<T>::mma(bf[j], af[i], acc[i][j]);
    }
    if (kt + 1 < KT) sstore((kt + 1) & 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wn * WTN + j * 16 + Mfma<T>::col(lane, r);
        if (row < M && col < N) C[row + col * ldc] = acc[i][j][r];
      }
    }
  }
}

// FP64 C -= A * B on v_mfma_f64_16x16x4f64: double-buffered LDS, peeled K
// loop, accumulators started from -C, interior tiles unmasked.  Each
// wavefront owns a WTM x WTN tile of 16x16 products (8 independent
// accumulators for the 64x32 tile of the 8-wavefront 128x128 launch, four
// wavefronts per SIMD).  The operands are passed swapped (B first), so each
// lane holds 16 consecutive rows of a column of C and the stores coalesce.
// V > 1: interior tiles of 16-byte aligned operands stage A and B with
// 16-byte loads (V rows of A, V k of B per thread: V = 2 for FP64, 4 for
// FP32); the k order of the products, hence every result bit, is the same
// for V = 1 and V > 1.  The same body serves FP32 on v_mfma_f32_16x16x4f32.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, bool EDGE, int V = 1>
__device__ __forceinline__ void gemm16_body(int64_t M, int64_t N, int64_t K, const T* __restrict__ A, int64_t lda,
                                            const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc,
                                            int64_t m0, int64_t n0, T* sA, T* sB) {
  typedef Mfma<T> MF;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int PAD = 16;  // 128-byte k-row runs, 1152 B apart: two bank passes, no extra conflict
  constexpr int LDSA = BM + PAD, LDSB = BN + PAD;
  constexpr int SA = BK * LDSA, SB = BK * LDSB;
  static_assert(V == 1 || (V * sizeof(T) == 16 && !EDGE), "16-byte staging on interior tiles only");
  constexpr int TA = BM / V, TB = BK / V;  // threads per k-row of A, per column of B
  constexpr int KA = NT / TA, NB_ = NT / TB;
  constexpr int EA = BK / KA, EB = BN / NB_;
  static_assert(KA * TA == NT && EA * KA == BK && NB_ * TB == NT && EB * NB_ == BN, "thread layout");
  typedef T VT __attribute__((ext_vector_type(V)));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  const int ai = (tid % TA) * V, ak0 = tid / TA;
  const int bk = (tid % TB) * V, bn0 = tid / TB;
  const bool arow_ok = !EDGE || (m0 + ai) < M;
  const T* pa = A + (arow_ok ? (m0 + ai) : (M - 1)) + (int64_t)ak0 * lda;
  const int64_t astep = (int64_t)KA * lda;
  bool bcol_ok[EB];
  const T* pb[EB];
#pragma unroll
  for (int s = 0; s < EB; ++s) {
    const int64_t gn = n0 + bn0 + NB_ * s;
    bcol_ok[s] = !EDGE || gn < N;
    pb[s] = B + (bcol_ok[s] ? gn : (N - 1)) * ldb + bk;
  }

  T ra[EA * V], rb[EB * V];
  auto gload = [&](int64_t k0) {
    if (V > 1) {
      const T* q = pa + k0 * lda;
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        const VT v = *reinterpret_cast<const VT*>(q + s * astep);
#pragma unroll
        for (int e = 0; e < V; ++e) ra[V * s + e] = v[e];
      }
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const VT v = *reinterpret_cast<const VT*>(pb[s] + k0);
#pragma unroll
        for (int e = 0; e < V; ++e) rb[V * s + e] = v[e];
      }
    } else if (!EDGE) {
      const T* q = pa + k0 * lda;
#pragma unroll
      for (int s = 0; s < EA; ++s) ra[s] = q[s * astep];
#pragma unroll
      for (int s = 0; s < EB; ++s) rb[s] = pb[s][k0];
    } else {
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        const int64_t gk = k0 + ak0 + KA * s;
        const int64_t gkc = gk < K ? gk : K - 1;
        const T v = pa[(gkc - ak0) * lda];
        ra[s] = (arow_ok && gk < K) ? v : T(0);
      }
      const int64_t gk = k0 + bk;
      const bool kok = gk < K;
      const int64_t off = (kok ? gk : K - 1) - bk;
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const T v = pb[s][off];
        rb[s] = (kok && bcol_ok[s]) ? v : T(0);
      }
    }
  };
  auto sstore = [&](int buf) {
    T* a = sA + buf * SA + ak0 * LDSA + ai;
    T* b = sB + buf * SB + bk * LDSB + bn0;
    if (V > 1) {
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        VT v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = ra[V * s + e];
        *reinterpret_cast<VT*>(a + s * KA * LDSA) = v;
      }
#pragma unroll
      for (int s = 0; s < EB; ++s)
#pragma unroll
        for (int e = 0; e < V; ++e) b[s * NB_ + e * LDSB] = rb[V * s + e];
    } else {
#pragma unroll
      for (int s = 0; s < EA; ++s) a[s * KA * LDSA] = ra[s];
#pragma unroll
      for (int s = 0; s < EB; ++s) b[s * NB_] = rb[s];
    }
  };

  const int lr = lane & 15, lk = lane >> 4;
  // accumulators from -C: lane holds rows lr of the 16x16 tile, column col(lane, q)
  typename MF::v4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + lr;
    const int64_t rowc = (!EDGE || row < M) ? row : M - 1;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + MF::col(lane, q);
        const int64_t colc = (!EDGE || col < N) ? col : N - 1;
        const T v = C[rowc + colc * ldc];
        acc[i][j][q] = (!EDGE || (row < M && col < N)) ? -v : T(0);
      }
  }

  auto compute = [&](int buf) {
    const T* as = sA + buf * SA + lk * LDSA + wm * WTM + lr;
    const T* bs = sB + buf * SB + lk * LDSB + wn * WTN + lr;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      T af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = as[kk * 4 * LDSA + i * 16];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = bs[kk * 4 * LDSB + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = MF::mma(bf[j], af[i], acc[i][j]);
    }
  };

  const int KT = (int)((K + BK - 1) / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt + 1 < KT; ++kt) {
    gload((int64_t)(kt + 1) * BK);
    compute(kt & 1);
    sstore((kt + 1) & 1);
    __syncthreads();
  }
  compute((KT - 1) & 1);

#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + lr;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + MF::col(lane, q);
        if (!EDGE || (row < M && col < N)) C[row + col * ldc] = -acc[i][j][q];
      }
  }
}

// Tile placement and the interior / edge / aligned dispatch of the gemm16
// kernels.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int GM>
__device__ __forceinline__ void gemm16_tile(int64_t M, int64_t N, int64_t K, const T* __restrict__ A, int64_t lda,
                                            const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc,
                                            int tiles_m, int tiles_n, T* sA, T* sB) {
  constexpr int V = 16 / (int)sizeof(T);
  const int total = tiles_m * tiles_n;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int bid = blockIdx.x;
  const int t = (bid % kXcds) * per_xcd + bid / kXcds;
  if (t >= total) return;
  const int group_size = GM * tiles_n;
  const int group = t / group_size;
  const int first_m = group * GM;
  const int gm = min(tiles_m - first_m, GM);
  const int within = t - group * group_size;
  const int tm = first_m + within % gm;
  const int tn = within / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const bool vec = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 && lda % V == 0 &&
                   ldb % V == 0;
  if (m0 + BM <= M && n0 + BN <= N && K % BK == 0) {
    if (vec)
      gemm16_body<T, BM, BN, BK, WGM, WGN, false, V>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sA, sB);
    else
      gemm16_body<T, BM, BN, BK, WGM, WGN, false, 1>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sA, sB);
  } else {
    gemm16_body<T, BM, BN, BK, WGM, WGN, true, 1>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sA, sB);
  }
}

// ROLE only names the launch: 0 for the trailing updates on the main and bulk
// streams, 1 for the share of the remaining-columns update run on the panel's
// CUs, 2 for the products inside the column-block and triangular-solve
// recursions.
template <int BM, int BN, int BK, int WGM, int WGN, int MINB, int ROLE, int GM = kGroupM>
__global__ __launch_bounds__(64 * WGM* WGN, MINB) void k_dgemm_sub_16(int64_t M, int64_t N, int64_t K,
                                                                      const double* __restrict__ A, int64_t lda,
                                                                      const double* __restrict__ B, int64_t ldb,
                                                                      double* __restrict__ C, int64_t ldc,
                                                                      int tiles_m, int tiles_n) {
  constexpr int PAD = 16;
  __shared__ __attribute__((aligned(16))) double sA[2 * BK * (BM + PAD)];
  __shared__ double sB[2 * BK * (BN + PAD)];
  gemm16_tile<double, BM, BN, BK, WGM, WGN, GM>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, sA, sB);
}

// FP32 C -= A * B on v_mfma_f32_16x16x4f32 with the same body (16-byte
// staging: four rows of A, four k of B per thread on interior tiles).
template <int BM, int BN, int BK, int WGM, int WGN, int MINB, int ROLE, int GM = kGroupM>
__global__ __launch_bounds__(64 * WGM* WGN, MINB) void k_sgemm_sub_16(int64_t M, int64_t N, int64_t K,
                                                                      const float* __restrict__ A, int64_t lda,
                                                                      const float* __restrict__ B, int64_t ldb,
                                                                      float* __restrict__ C, int64_t ldc,
                                                                      int tiles_m, int tiles_n) {
  constexpr int PAD = 16;
  __shared__ __attribute__((aligned(16))) float sA[2 * BK * (BM + PAD)];
  __shared__ float sB[2 * BK * (BN + PAD)];
  gemm16_tile<float, BM, BN, BK, WGM, WGN, GM>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, sA, sB);
}

namespace {

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int MINB>
hipError_t launch(hipStream_t s, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                  int64_t ldb, T* C, int64_t ldc) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  if (tm * tn > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL((k_gemm_sub<T, BM, BN, BK, WGM, WGN, MINB>), dim3(per_xcd * kXcds), dim3(64 * WGM * WGN), 0,
                     s, M, N, K, A, lda, B, ldb, C, ldc, (int)tm, (int)tn);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WGM, int WGN, int MINB, int ROLE = 0, int GM = kGroupM>
hipError_t launch_d16(hipStream_t s, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  if (tm * tn > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL((k_dgemm_sub_16<BM, BN, BK, WGM, WGN, MINB, ROLE, GM>), dim3(per_xcd * kXcds), dim3(64 * WGM * WGN), 0,
                     s, M, N, K, A, lda, B, ldb, C, ldc, (int)tm, (int)tn);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WGM, int WGN, int MINB, int ROLE = 0, int GM = kGroupM>
hipError_t launch_s16(hipStream_t s, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                      int64_t ldb, float* C, int64_t ldc) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  if (tm * tn > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL((k_sgemm_sub_16<BM, BN, BK, WGM, WGN, MINB, ROLE, GM>), dim3(per_xcd * kXcds),
                     dim3(64 * WGM * WGN), 0, s, M, N, K, A, lda, B, ldb, C, ldc, (int)tm, (int)tn);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t gemm_sub(hipStream_t s, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                    int64_t ldb, T* C, int64_t ldc, int* tile_out, int role) {
  int dummy;
  int& tile = tile_out ? *tile_out : dummy;
  tile = -1;
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (N <= 32) {
    tile = 0;
    return launch<T, 128, 32, 16, 4, 1, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
  }
  const int64_t big_tiles = ((M + 127) / 128) * ((N + 127) / 128);
  if constexpr (sizeof(T) == 8) {
    if (big_tiles >= 256 || (role == 1 && big_tiles >= 32)) {
      tile = 1;
      if (role == 1) return launch_d16<128, 128, 8, 2, 4, 4, 1>(s, M, N, K, A, lda, B, ldb, C, ldc);
      if (role == 2) return launch_d16<128, 128, 8, 2, 4, 4, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
      return launch_d16<128, 128, 8, 2, 4, 4>(s, M, N, K, A, lda, B, ldb, C, ldc);
    }
    tile = 2;
    return launch_d16<64, 64, 8, 2, 2, 4>(s, M, N, K, A, lda, B, ldb, C, ldc);
  } else {
    if (big_tiles >= 512 || (role == 1 && big_tiles >= 32)) {
      tile = 1;
      if (role == 1) return launch_s16<128, 128, 16, 2, 2, 2, 1>(s, M, N, K, A, lda, B, ldb, C, ldc);
      if (role == 2) return launch_s16<128, 128, 16, 2, 2, 2, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
      return launch_s16<128, 128, 16, 2, 2, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
    }
    tile = 2;
    if (role == 1) return launch_s16<64, 64, 16, 2, 2, 4, 1>(s, M, N, K, A, lda, B, ldb, C, ldc);
    if (role == 2) return launch_s16<64, 64, 16, 2, 2, 4, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
    return launch_s16<64, 64, 16, 2, 2, 4>(s, M, N, K, A, lda, B, ldb, C, ldc);
  }
}

template hipError_t gemm_sub<double>(hipStream_t, int64_t, int64_t, int64_t, const double*, int64_t,
                                     const double*, int64_t, double*, int64_t, int*, int);
template hipError_t gemm_sub<float>(hipStream_t, int64_t, int64_t, int64_t, const float*, int64_t,
                                    const float*, int64_t, float*, int64_t, int*, int);

}  // namespace lupp
