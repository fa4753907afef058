// Low-precision trailing update for the mixed-precision factorization:
//   C (FP32) -= A (FP32) * B (FP32)
// with A and B rounded to BF16, FP16 or FP8 (OCP e4m3) while they are staged
// into LDS, products on v_mfma_f32_16x16x32_{bf16,f16,fp8_fp8} and FP32
// accumulation.  This is the matrix-matrix product that dominates the
// factorization (the paper's Sections 4.1 and 5.4), carried out in a cheaper
// format; the FP64 refinement wins the accuracy back.
//
// Scaling: the operands of FP16 and FP8 would under- or overflow (multipliers
// of L21 shrink like 1/n for diagonally dominant matrices; e4m3's largest
// value is 448), so each 128-row block of A and each 128-column block of B is
// multiplied by a power of two 2^e chosen from its largest magnitude (exact:
// only the exponent changes) before rounding.  One tile of C then carries one
// scale 2^(ea+eb): the MFMAs accumulate the scaled products from zero and the
// epilogue stores C - (acc * 2^-ea) * 2^-eb (C itself is loaded into registers
// during the last K step so that its latency hides behind the final products;
// it is never scaled, so no magnitude of C can overflow).  BF16 has FP32's exponent range
// and uses no scaling.
//
// Two ways to stage the operands, with the same rounded values and the same
// order of products (hence the same result bits):
//  - packed (default): A and B are scaled and rounded once per update into
//    a workspace laid out in MFMA fragment order (k_lp_pack_a, k_lp_pack_b);
//    the GEMM (k_gemm_lpq) then loads each lane's 8-element operand with one
//    coalesced load, with no LDS, no barrier and no per-tile conversion;
//  - staged: each tile converts its FP32 operands while copying them into
//    LDS (k_gemm_lp); used when no packing workspace fits the call.
//
// Lane layout of the 16x16x32 instructions (probed on gfx950): lane l supplies
// A(l%16, 8*(l/16)+t) and B(8*(l/16)+t, l%16), t = 0..7.  The operands are
// passed swapped (B as the first), so lane l receives C(l%16, 4*(l/16)+r):
// sixteen consecutive rows of a column per register, coalesced stores.
#include "common.h"

namespace lupp {

namespace {

constexpr int kXcdsLp = 8;
constexpr int kGroupMLp = 8;
constexpr int BM = 128, BN = 128, BK = 32, NT = 256;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

template <int MODE>
struct Lp;

// MODE 1: BF16
template <>
struct Lp<1> {
  static constexpr int kBytes = 16;  // bytes of one lane's 8-element operand
  typedef uint4 packed;
  static __device__ __forceinline__ packed pack(const float* v) {
    bf8 b;  // v_cvt_pk_bf16_f32: round to nearest even
#pragma unroll
    for (int t = 0; t < 8; ++t) b[t] = (__bf16)v[t];
    return __builtin_bit_cast(uint4, b);
  }
  static __device__ __forceinline__ f4 mma(packed a, packed b, f4 c) {
    bf8 av = __builtin_bit_cast(bf8, a), bv = __builtin_bit_cast(bf8, b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};

// MODE 2: FP16
template <>
struct Lp<2> {
  static constexpr int kBytes = 16;
  typedef uint4 packed;
  static __device__ __forceinline__ packed pack(const float* v) {
    h8 h;
#pragma unroll
    for (int t = 0; t < 8; ++t) h[t] = (_Float16)v[t];
    return __builtin_bit_cast(uint4, h);
  }
  static __device__ __forceinline__ f4 mma(packed a, packed b, f4 c) {
    h8 av = __builtin_bit_cast(h8, a), bv = __builtin_bit_cast(h8, b);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
};

// MODE 3: FP8 (OCP e4m3, saturating conversion)
template <>
struct Lp<3> {
  static constexpr int kBytes = 8;
  typedef uint2 packed;
  static __device__ __forceinline__ packed pack(const float* v) {
    int lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], hi, true);
    return make_uint2((uint32_t)lo, (uint32_t)hi);
  }
  static __device__ __forceinline__ f4 mma(packed a, packed b, f4 c) {
    const long av = (long)(((uint64_t)a.y << 32) | a.x), bv = (long)(((uint64_t)b.y << 32) | b.x);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, c, 0, 0, 0);
  }
};

template <int MODE>
__global__ __launch_bounds__(NT, 2) void k_gemm_lp(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                                   int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                   float* __restrict__ C, int64_t ldc, const int* __restrict__ ea,
                                                   const int* __restrict__ eb, int tiles_m, int tiles_n) {
  typedef Lp<MODE> L;
  typedef typename L::packed P;
  constexpr int RB = L::kBytes * (BK / 8) + 16;  // LDS row bytes (padded)
  constexpr int WGM = 2, WTM = BM / WGM, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
  __shared__ __attribute__((aligned(16))) unsigned char sA[2][BM * RB];
  __shared__ __attribute__((aligned(16))) unsigned char sB[2][BN * RB];

  const int total = tiles_m * tiles_n;
  const int per_xcd = (total + kXcdsLp - 1) / kXcdsLp;
  const int bid = blockIdx.x;
  const int t = (bid % kXcdsLp) * per_xcd + bid / kXcdsLp;
  if (t >= total) return;
  const int group_size = kGroupMLp * tiles_n;
  const int group = t / group_size;
  const int first_m = group * kGroupMLp;
  const int gm = min(tiles_m - first_m, kGroupMLp);
  const int within = t - group * group_size;
  const int tm = first_m + within % gm;
  const int tn = within / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  const int sea = ea ? ea[tm] : 0, seb = eb ? eb[tn] : 0;
  const float fa = ldexpf(1.0f, sea), fb = ldexpf(1.0f, seb);
  const float fai = ldexpf(1.0f, -sea), fbi = ldexpf(1.0f, -seb);

  // staging of A: thread owns rows 2*ra2, 2*ra2 + 1 and the k-group ka (one
  // 8-byte load per k; a load instruction reads 512 consecutive bytes of a
  // column).  Staging of B: four threads share a column; thread tid takes
  // column cb0 (and cb0 + 64) and the k-group kb (two 16-byte loads; one load
  // instruction covers 16 whole column segments).  Loads keep the raw values;
  // rows, columns and k out of range are masked while staging to LDS, so no
  // load result is consumed before the products of the step.
  const int ra2 = tid & 63, ka = tid >> 6;
  const int cb0 = tid >> 2, kb = tid & 3;
  const bool arow0 = (m0 + 2 * ra2) < M, arow1 = (m0 + 2 * ra2 + 1) < M;
  const bool bcol0 = (n0 + cb0) < N, bcol1 = (n0 + cb0 + 64) < N;
  // a pair straddling row M - 1 (M odd) is read as rows M - 2, M - 1
  const int64_t ar = (m0 + 2 * ra2 + 1 < M) ? (m0 + 2 * ra2) : (M >= 2 ? M - 2 : 0);
  const bool apair = M >= 2;
  const float* pa = A + ar;
  const float* pb0 = B + (bcol0 ? (n0 + cb0) : (N - 1)) * ldb;
  const float* pb1 = B + (bcol1 ? (n0 + cb0 + 64) : (N - 1)) * ldb;
  // which of the two loaded rows holds row 2*ra2 (only differs when shifted)
  const bool ashift = (m0 + 2 * ra2 + 1 >= M) && apair && (m0 + 2 * ra2 < M);

  float va[2][8], vb[2][8];
  auto gload = [&](int64_t k0) {
    if (k0 + BK <= K) {
      if (apair) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const f2u x = *(const f2u*)(pa + (k0 + 8 * ka + q) * lda);
          va[0][q] = x[0];
          va[1][q] = x[1];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) va[0][q] = va[1][q] = pa[(k0 + 8 * ka + q) * lda];
      }
      const f4u b00 = *(const f4u*)(pb0 + k0 + 8 * kb), b01 = *(const f4u*)(pb0 + k0 + 8 * kb + 4);
      const f4u b10 = *(const f4u*)(pb1 + k0 + 8 * kb), b11 = *(const f4u*)(pb1 + k0 + 8 * kb + 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        vb[0][q] = b00[q];
        vb[0][q + 4] = b01[q];
        vb[1][q] = b10[q];
        vb[1][q + 4] = b11[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = k0 + 8 * ka + q;
        const int64_t kc = k < K ? k : K - 1;
        va[0][q] = pa[kc * lda];
        va[1][q] = pa[kc * lda + (apair ? 1 : 0)];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = k0 + 8 * kb + q;
        const int64_t kc = k < K ? k : K - 1;
        vb[0][q] = pb0[kc];
        vb[1][q] = pb1[kc];
      }
    }
  };
  auto sstore = [&](int buf, int64_t k0) {
    const int64_t kab = k0 + 8 * ka, kbb = k0 + 8 * kb;
    float x0[8], x1[8], y0[8], y1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool kin = kab + q < K;
      const float r0 = ashift ? va[1][q] : va[0][q];
      x0[q] = (arow0 && kin) ? r0 * fa : 0.0f;
      x1[q] = (arow1 && kin) ? va[1][q] * fa : 0.0f;
      const bool kin2 = kbb + q < K;
      y0[q] = (bcol0 && kin2) ? vb[0][q] * fb : 0.0f;
      y1[q] = (bcol1 && kin2) ? vb[1][q] * fb : 0.0f;
    }
    *(P*)(sA[buf] + (2 * ra2) * RB + ka * L::kBytes) = L::pack(x0);
    *(P*)(sA[buf] + (2 * ra2 + 1) * RB + ka * L::kBytes) = L::pack(x1);
    *(P*)(sB[buf] + cb0 * RB + kb * L::kBytes) = L::pack(y0);
    *(P*)(sB[buf] + (cb0 + 64) * RB + kb * L::kBytes) = L::pack(y1);
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  const int koff = (lane >> 4) * L::kBytes;
  auto products = [&](int buf) {
    P af[FM], bf[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) af[i] = *(const P*)(sA[buf] + (wm * WTM + i * 16 + (lane & 15)) * RB + koff);
#pragma unroll
    for (int j = 0; j < FN; ++j) bf[j] = *(const P*)(sB[buf] + (wn * WTN + j * 16 + (lane & 15)) * RB + koff);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = L::mma(bf[j], af[i], acc[i][j]);
  };

  const int KT = (int)((K + BK - 1) / BK);
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt + 1 < KT; ++kt) {
    const int64_t kn = (int64_t)(kt + 1) * BK;
    gload(kn);
    products(kt & 1);
    sstore((kt + 1) & 1, kn);
    __syncthreads();
  }
  // last K step: the staging registers are free, so C is loaded here and its
  // latency overlaps the final products
  f4 cpre[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
    const int64_t rowc = row < M ? row : M - 1;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + q;
        const int64_t colc = col < N ? col : N - 1;
        cpre[i][j][q] = C[rowc + colc * ldc];
      }
  }
  products((KT - 1) & 1);

#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + q;
        if (row < M && col < N) C[row + col * ldc] = cpre[i][j][q] - (acc[i][j][q] * fai) * fbi;
      }
  }
}

// Packed operands: for each 128-row block of A (128-column block of B) and
// each 32-deep chunk of k, 128 rows of 32 rounded values, row-major (ROWB
// bytes per row; the 8 values a lane supplies for k-group g sit at byte
// offset g * kBytes of the row).  Rows, columns and k out of range are zero.
template <int MODE>
constexpr int lp_rowb() {
  return 4 * Lp<MODE>::kBytes;
}

// A (FP32, column-major M x K) scaled by 2^ea[block] and rounded; one
// workgroup per (128-row block, 32-deep chunk).  Thread c of 512 chunks takes
// row c % 128 and k-group c / 128, so each of its 8 loads reads 64
// consecutive rows of one column across the wavefront.
template <int MODE>
__global__ __launch_bounds__(256) void k_lp_pack_a(int64_t M, int64_t K, const float* __restrict__ A, int64_t lda,
                                                   const int* __restrict__ ea, int KC,
                                                   unsigned char* __restrict__ out) {
  typedef Lp<MODE> L;
  constexpr int ROWB = lp_rowb<MODE>();
  const int tm = blockIdx.x, kc = blockIdx.y;
  const float f = ea ? ldexpf(1.0f, ea[tm]) : 1.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = threadIdx.x + 256 * h;
    const int row = c & 127, g = c >> 7;
    const int64_t gr = (int64_t)tm * 128 + row;
    const int64_t k0 = (int64_t)kc * 32 + 8 * g;
    // loads at indices clamped into A, then the selects (a guarded load per
    // value would wait for the one before it)
    const int64_t grc = gr < M ? gr : M - 1;
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t k = k0 + t;
      v[t] = A[grc + (k < K ? k : K - 1) * lda];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (gr < M && k0 + t < K) ? v[t] * f : 0.0f;
    *(typename L::packed*)(out + ((size_t)((int64_t)tm * KC + kc) * 128 + row) * ROWB + g * L::kBytes) =
        L::pack(v);
  }
}

// B (FP32, column-major K x N) scaled by 2^eb[block] and rounded; one
// workgroup per (128-column block, 32-deep chunk).  Four threads share a
// column (k-groups 0..3), so a column's 32 values are read together.
template <int MODE>
__global__ __launch_bounds__(256) void k_lp_pack_b(int64_t K, int64_t N, const float* __restrict__ B, int64_t ldb,
                                                   const int* __restrict__ eb, int KC,
                                                   unsigned char* __restrict__ out) {
  typedef Lp<MODE> L;
  constexpr int ROWB = lp_rowb<MODE>();
  const int tn = blockIdx.x, kc = blockIdx.y;
  const float f = eb ? ldexpf(1.0f, eb[tn]) : 1.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = threadIdx.x + 256 * h;
    const int g = c & 3, col = c >> 2;
    const int64_t gc = (int64_t)tn * 128 + col;
    const int64_t k0 = (int64_t)kc * 32 + 8 * g;
    const int64_t gcc = gc < N ? gc : N - 1;
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t k = k0 + t;
      v[t] = B[(k < K ? k : K - 1) + gcc * ldb];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (gc < N && k0 + t < K) ? v[t] * f : 0.0f;
    *(typename L::packed*)(out + ((size_t)((int64_t)tn * KC + kc) * 128 + col) * ROWB + g * L::kBytes) =
        L::pack(v);
  }
}

// C (FP32) -= A * B from packed operands: 128 x 128 tiles, four wavefronts of
// 64 x 64 (16 accumulators), each lane loading its own fragments straight
// from the packed chunks (one 16-byte load per fragment for BF16/FP16, 8 for
// FP8), two chunks in flight.  C is loaded at the start (its latency hides
// behind the products) and stored once, unscaled: C - (acc 2^-ea) 2^-eb.
template <int MODE>
__global__ __launch_bounds__(NT, 2) void k_gemm_lpq(int64_t M, int64_t N, int KC,
                                                    const unsigned char* __restrict__ Aq,
                                                    const unsigned char* __restrict__ Bq, float* __restrict__ C,
                                                    int64_t ldc, const int* __restrict__ ea,
                                                    const int* __restrict__ eb, int tiles_m, int tiles_n) {
  typedef Lp<MODE> L;
  typedef typename L::packed P;
  constexpr int ROWB = lp_rowb<MODE>();
  constexpr int CH = 128 * ROWB;  // bytes of one 32-deep chunk of a 128-row block
  constexpr int WGM = 2, WTM = BM / WGM, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;

  const int total = tiles_m * tiles_n;
  const int per_xcd = (total + kXcdsLp - 1) / kXcdsLp;
  const int bid = blockIdx.x;
  const int t = (bid % kXcdsLp) * per_xcd + bid / kXcdsLp;
  if (t >= total) return;
  const int group_size = kGroupMLp * tiles_n;
  const int group = t / group_size;
  const int first_m = group * kGroupMLp;
  const int gm = min(tiles_m - first_m, kGroupMLp);
  const int within = t - group * group_size;
  const int tm = first_m + within % gm;
  const int tn = within / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  const int sea = ea ? ea[tm] : 0, seb = eb ? eb[tn] : 0;
  const float fai = ldexpf(1.0f, -sea), fbi = ldexpf(1.0f, -seb);

  const unsigned char* pa =
      Aq + (size_t)tm * KC * CH + (wm * WTM + (lane & 15)) * ROWB + (lane >> 4) * L::kBytes;
  const unsigned char* pb =
      Bq + (size_t)tn * KC * CH + (wn * WTN + (lane & 15)) * ROWB + (lane >> 4) * L::kBytes;

  f4 cpre[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
    const int64_t rowc = row < M ? row : M - 1;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + q;
        const int64_t colc = col < N ? col : N - 1;
        cpre[i][j][q] = C[rowc + colc * ldc];
      }
  }

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  P a0[FM], b0[FN], a1[FM], b1[FN];
  auto load = [&](int kc, P* a, P* b) {
#pragma unroll
    for (int i = 0; i < FM; ++i) a[i] = *(const P*)(pa + (size_t)kc * CH + i * 16 * ROWB);
#pragma unroll
    for (int j = 0; j < FN; ++j) b[j] = *(const P*)(pb + (size_t)kc * CH + j * 16 * ROWB);
  };
  auto products = [&](const P* a, const P* b) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = L::mma(b[j], a[i], acc[i][j]);
  };

  load(0, a0, b0);
  int kc = 0;
  for (; kc + 2 <= KC; kc += 2) {
    load(kc + 1, a1, b1);
    products(a0, b0);
    if (kc + 2 < KC) load(kc + 2, a0, b0);
    products(a1, b1);
  }
  if (kc < KC) products(a0, b0);

#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int64_t row = m0 + wm * WTM + i * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + q;
        if (row < M && col < N) C[row + col * ldc] = cpre[i][j][q] - (acc[i][j][q] * fai) * fbi;
      }
  }
}

// wavefront max of floats, the same value in every lane
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// exponent e of each 128-row block of A (dim = 0) or 128-column block of B
// (dim = 1) such that 2^e * max|block| lies in [limit/2, limit]; 0 for a zero
// block.  limit is the format's largest finite value.  1024 threads per
// block, each keeping four loads in flight; every load instruction reads 64
// consecutive elements of a column.  (The maximum does not depend on the
// order it is taken in: fmaxf is exact and skips NaN either way.)
__global__ __launch_bounds__(1024) void k_block_exp(int64_t rows, int64_t cols, const float* __restrict__ X,
                                                    int64_t ldx, int dim, float limit, int* __restrict__ e) {
  __shared__ float s_max[16];
  const int blk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float m = 0.0f;
  if (dim == 0) {
    // rows r0 + (tid & 127), columns tid >> 7, + 8, + 16, ...
    const int64_t r = (int64_t)blk * 128 + (tid & 127);
    if (r < rows) {
      const float* p = X + r;
      int64_t c = tid >> 7;
      for (; c + 24 < cols; c += 32) {
        const float a0 = p[c * ldx], a1 = p[(c + 8) * ldx], a2 = p[(c + 16) * ldx], a3 = p[(c + 24) * ldx];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(a0), fabsf(a1)), fmaxf(fabsf(a2), fabsf(a3))));
      }
      for (; c < cols; c += 8) m = fmaxf(m, fabsf(p[c * ldx]));
    }
  } else {
    // columns c0 + 8 * wave .. + 7, rows lane, lane + 64, ...
    for (int cc = 0; cc < 8; ++cc) {
      const int64_t c = (int64_t)blk * 128 + wave * 8 + cc;
      if (c >= cols) break;
      const float* p = X + c * ldx;
      int64_t r = lane;
      for (; r + 192 < rows; r += 256) {
        const float a0 = p[r], a1 = p[r + 64], a2 = p[r + 128], a3 = p[r + 192];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(a0), fabsf(a1)), fmaxf(fabsf(a2), fabsf(a3))));
      }
      for (; r < rows; r += 64) m = fmaxf(m, fabsf(p[r]));
    }
  }
  m = wave_max(m);
  if (lane == 0) s_max[wave] = m;
  __syncthreads();
  if (tid == 0) {
    float mx = 0.0f;
    for (int w = 0; w < 16; ++w) mx = fmaxf(mx, s_max[w]);
    int ex = 0;
    if (mx > 0.0f && mx < 3.0e38f) {
      (void)frexpf(limit / mx, &ex);  // limit/mx = f * 2^ex, f in [0.5, 1)
      ex -= 1;                        // 2^ex <= limit/mx
      ex = ex > 100 ? 100 : (ex < -100 ? -100 : ex);
    }
    e[blk] = ex;
  }
}

template <int MODE>
hipError_t launch_lp(hipStream_t s, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                     int64_t ldb, float* C, int64_t ldc, const int* ea, const int* eb) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  if (tm * tn > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcdsLp - 1) / kXcdsLp;
  hipLaunchKernelGGL((k_gemm_lp<MODE>), dim3(per_xcd * kXcdsLp), dim3(NT), 0, s, M, N, K, A, lda, B, ldb, C, ldc, ea,
                     eb, (int)tm, (int)tn);
  return hipGetLastError();
}

// Packs A and B into `pack` (gemm_lp_pack_bytes(M, N, K) bytes) and runs the
// packed GEMM.
template <int MODE>
hipError_t launch_lpq(hipStream_t s, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                      int64_t ldb, float* C, int64_t ldc, const int* ea, const int* eb, unsigned char* pack) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN, kc = (K + 31) / 32;
  if (tm * tn > (int64_t)1 << 30 || kc > 65535 || tm > 0x7fffffff || tn > 0x7fffffff) return hipErrorInvalidValue;
  unsigned char* aq = pack;
  unsigned char* bq = pack + (size_t)tm * kc * 128 * lp_rowb<MODE>();
  hipLaunchKernelGGL(k_lp_pack_a<MODE>, dim3((unsigned)tm, (unsigned)kc), dim3(256), 0, s, M, K, A, lda, ea, (int)kc,
                     aq);
  hipLaunchKernelGGL(k_lp_pack_b<MODE>, dim3((unsigned)tn, (unsigned)kc), dim3(256), 0, s, K, N, B, ldb, eb, (int)kc,
                     bq);
  const int total = (int)(tm * tn);
  const int per_xcd = (total + kXcdsLp - 1) / kXcdsLp;
  hipLaunchKernelGGL((k_gemm_lpq<MODE>), dim3(per_xcd * kXcdsLp), dim3(NT), 0, s, M, N, (int)kc, aq, bq, C, ldc, ea,
                     eb, (int)tm, (int)tn);
  return hipGetLastError();
}

}  // namespace

int64_t gemm_lp_scale_slots(int64_t M, int64_t N) { return (M + BM - 1) / BM + (N + BN - 1) / BN; }

size_t gemm_lp_pack_bytes(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN, kc = (K + 31) / 32;
  return (size_t)(tm + tn) * (size_t)kc * 128 * (size_t)lp_rowb<1>();  // BF16/FP16 rows; FP8 uses half
}

hipError_t gemm_lp_sub(hipStream_t s, int mode, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float* C, int64_t ldc, int* scale_ws, void* pack,
                       size_t pack_bytes) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (mode < 1 || mode > 3) return hipErrorInvalidValue;
  const bool packed = pack && gemm_lp_pack_bytes(M, N, K) <= pack_bytes;
  unsigned char* pk = (unsigned char*)pack;
  if (mode == 1)
    return packed ? launch_lpq<1>(s, M, N, K, A, lda, B, ldb, C, ldc, nullptr, nullptr, pk)
                  : launch_lp<1>(s, M, N, K, A, lda, B, ldb, C, ldc, nullptr, nullptr);
  const float limit = (mode == 2) ? 65504.0f : 448.0f;
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  int* ea = scale_ws;
  int* eb = scale_ws + tm;
  hipLaunchKernelGGL(k_block_exp, dim3((unsigned)tm), dim3(1024), 0, s, M, K, A, lda, 0, limit, ea);
  hipLaunchKernelGGL(k_block_exp, dim3((unsigned)tn), dim3(1024), 0, s, K, N, B, ldb, 1, limit, eb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == 2)
    return packed ? launch_lpq<2>(s, M, N, K, A, lda, B, ldb, C, ldc, ea, eb, pk)
                  : launch_lp<2>(s, M, N, K, A, lda, B, ldb, C, ldc, ea, eb);
  return packed ? launch_lpq<3>(s, M, N, K, A, lda, B, ldb, C, ldc, ea, eb, pk)
                : launch_lp<3>(s, M, N, K, A, lda, B, ldb, C, ldc, ea, eb);
}

}  // namespace lupp
