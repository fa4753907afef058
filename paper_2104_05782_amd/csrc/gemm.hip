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
// before the current step's MFMAs).  A is negated while it is staged, so the
// accumulators hold -A*B and the epilogue is a single read-add-write of C.
// Tiles are mapped XCD-aware: consecutive workgroup ids land on different XCDs
// (round robin), so the id is first split into (xcd, slot) and each XCD walks
// its own contiguous band of tiles in groups of 8 tile-rows, keeping the A
// rows and B columns it needs in its own L2.
#include "common.h"

namespace lupp {
namespace {

constexpr int kXcds = 8;
constexpr int kGroupM = 8;

template <typename T, int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM* WGN) void k_gemm_sub(int64_t M, int64_t N, int64_t K,
                                                            const T* __restrict__ A, int64_t lda,
                                                            const T* __restrict__ B, int64_t ldb,
                                                            T* __restrict__ C, int64_t ldc, int tiles_m,
                                                            int tiles_n) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int PAD = 16;
  constexpr int LDSA = BM + PAD, LDSB = BN + PAD;
  constexpr int EA = BM * BK / NT, EB = BK * BN / NT;
  static_assert(EA * NT == BM * BK && EB * NT == BK * BN, "tile/thread mismatch");
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

  T ra[EA], rb[EB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int s = 0; s < EA; ++s) {
      const int e = tid + NT * s;
      const int i = e % BM, k = e / BM;
      const int64_t gi = m0 + i, gk = k0 + k;
      ra[s] = (gi < M && gk < K) ? A[gi + gk * lda] : T(0);
    }
#pragma unroll
    for (int s = 0; s < EB; ++s) {
      const int e = tid + NT * s;
      const int k = e % BK, n = e / BK;
      const int64_t gk = k0 + k, gn = n0 + n;
      rb[s] = (gk < K && gn < N) ? B[gk + gn * ldb] : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < EA; ++s) {
      const int e = tid + NT * s;
      sA[buf][(e / BM) * LDSA + (e % BM)] = -ra[s];
    }
#pragma unroll
    for (int s = 0; s < EB; ++s) {
      const int e = tid + NT * s;
      sB[buf][(e % BK) * LDSB + (e / BK)] = rb[s];
    }
  };

  v4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4{0, 0, 0, 0};

  const int KT = (int)((K + BK - 1) / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    if (kt + 1 < KT) gload((int64_t)(kt + 1) * BK);
    const T* as = sA[kt & 1];
    const T* bs = sB[kt & 1];
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      T af[FM], bf[FN];
      const int krow = kk * 4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = as[krow * LDSA + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = bs[krow * LDSB + wn * WTN + j * 16 + (lane & 15)];
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
        if (row < M && col < N) {
          T* p = C + row + col * ldc;
          *p = *p + acc[i][j][r];
        }
      }
    }
  }
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch(hipStream_t s, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                  int64_t ldb, T* C, int64_t ldc) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  if (tm * tn > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL((k_gemm_sub<T, BM, BN, BK, WGM, WGN>), dim3(per_xcd * kXcds), dim3(64 * WGM * WGN), 0, s,
                     M, N, K, A, lda, B, ldb, C, ldc, (int)tm, (int)tn);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t gemm_sub(hipStream_t s, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                    int64_t ldb, T* C, int64_t ldc, int* tile_out) {
  int dummy;
  int& tile = tile_out ? *tile_out : dummy;
  tile = -1;
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (N <= 32) {
    tile = 0;
    return launch<T, 128, 32, 16, 4, 1>(s, M, N, K, A, lda, B, ldb, C, ldc);
  }
  const int64_t big_tiles = ((M + 127) / 128) * ((N + 127) / 128);
  if (big_tiles >= 512) {
    tile = 1;
    return launch<T, 128, 128, 16, 2, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
  }
  tile = 2;
  return launch<T, 64, 64, 16, 2, 2>(s, M, N, K, A, lda, B, ldb, C, ldc);
}

template hipError_t gemm_sub<double>(hipStream_t, int64_t, int64_t, int64_t, const double*, int64_t,
                                     const double*, int64_t, double*, int64_t, int*);
template hipError_t gemm_sub<float>(hipStream_t, int64_t, int64_t, int64_t, const float*, int64_t,
                                    const float*, int64_t, float*, int64_t, int*);

}  // namespace lupp
