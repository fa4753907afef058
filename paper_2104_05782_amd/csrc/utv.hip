// Randomized UTV factorization (randUTV, the paper's Section 3.2): A = U T V^T
// for a square A, U and V orthogonal, T upper triangular, built b = 64 columns
// at a time.  Step i (k0 = i b, T22 = T[k0:, k0:]):
//   V_alpha: Y = (T22^T T22)^q T22^T G_i (matrix products: G_i^T T22 and
//            P^T T22 on the transposed-product kernel of the QR path, T22 Y on
//            the GEMM), then the Householder QR of Y; T[:, k0:] and V[:, k0:]
//            are multiplied by its Q from the right;
//   U_alpha: the Householder QR of T22's first b columns, applied to the rest
//            of T22 (the QR path's outer block), and U[:, k0:] times its Q;
//   U_beta, V_beta: the SVD of the b x b diagonal block (one-sided Jacobi in
//            one workgroup), which becomes diag(sigma); Us^T and Vs go to the
//            block row and column of T, Us to U, Vs to V.
// Products with Q = I - V T V^T from the right are X Q = X - ((X V) T) V^T,
// three GEMMs.  The Gaussian draws are an input (G, n x n: step i uses
// G[k0:, k0:k0+b]), so the method's random numbers come from the caller.
#include "handle.h"
#include "wave.h"

namespace lupp {

namespace {

constexpr int kUtvB = 64;  // block size b
constexpr int kUtvMaxSweeps = 40;

// dst (cols x rows, ldd) = scale * src^T (src rows x cols, lds)
__global__ void k_utv_transpose(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                                double* __restrict__ dst, int64_t ldd, double scale) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows of 32
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    t[j][tx] = (r < rows && c < cols) ? src[r + c * lds] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + tx, r = r0 + j;  // dst(c, r) = src(r, c)
    if (r < rows && c < cols) dst[c + r * ldd] = scale * t[tx][j];
  }
}

// dst (rows x cols) = scale * src
__global__ void k_utv_scale_copy(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                                 double* __restrict__ dst, int64_t ldd, double scale) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % rows, c = e / rows;
    dst[r + c * ldd] = scale * src[r + c * lds];
  }
}

__global__ void k_utv_fill(int64_t rows, int64_t cols, double* __restrict__ x, int64_t ld, double v) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    x[e % rows + (e / rows) * ld] = v;
}

// the strictly lower part of the first w columns of a rows x w block := 0
__global__ void k_utv_zero_lower(int64_t rows, int w, double* __restrict__ x, int64_t ld) {
  const int64_t total = rows * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % rows, c = e / rows;
    if (r > c) x[r + c * ld] = 0.0;
  }
}

// The w x w block (w <= 64) := diag(sigma)
__global__ void k_utv_set_diag(int w, const double* __restrict__ sigma, double* __restrict__ x, int64_t ld) {
  for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
    const int r = e % w, c = e / w;
    x[r + (int64_t)c * ld] = (r == c) ? sigma[r] : 0.0;
  }
}

// Sum over the 64 lanes, the same value in every lane: pairs, quads, 8- and
// 16-lane mirrors by DPP (ALU latency, no LDS crossbar), then the four row
// sums read as scalars.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sums over the 64 lanes of a and b together.  After one exchange of each
// (lane pairs), even lanes carry a's partial sums and odd lanes b's, so the
// rest of the butterfly runs once for both: quads and the two row rotations
// (DPP, they keep a lane's parity), then the row pairs and the wave halves by
// the permlane swaps (v_permlane16_swap exchanges the odd rows of its first
// operand with the even rows of its second, v_permlane32_swap the upper half
// of the first with the lower half of the second: with both operands x, the
// two results add up to the sum of partners 16, resp. 32, apart).  a's sum is
// then in lane 0, b's in lane 1; both are returned to every lane.
__device__ __forceinline__ double join_u32(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double swap16_sum(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)(uint32_t)u, (int)(uint32_t)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(uint32_t)(u >> 32), (int)(uint32_t)(u >> 32), false, false);
  return join_u32((uint32_t)lo[0], (uint32_t)hi[0]) + join_u32((uint32_t)lo[1], (uint32_t)hi[1]);
}
__device__ __forceinline__ double swap32_sum(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)(uint32_t)u, (int)(uint32_t)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(uint32_t)(u >> 32), (int)(uint32_t)(u >> 32), false, false);
  return join_u32((uint32_t)lo[0], (uint32_t)hi[0]) + join_u32((uint32_t)lo[1], (uint32_t)hi[1]);
}
__device__ __forceinline__ void wave_sum2(double a, double b, int lane, double& sa, double& sb) {
  a += dpp_f64<0xB1>(a);  // lane ^ 1
  b += dpp_f64<0xB1>(b);
  double x = (lane & 1) ? b : a;
  x += dpp_f64<0x4E>(x);   // lane ^ 2
  x += dpp_f64<0x124>(x);  // row rotation by 4
  x += dpp_f64<0x128>(x);  // row rotation by 8
  x = swap16_sum(x);
  x = swap32_sum(x);
  sa = readlane_d(x, 0);
  sb = readlane_d(x, 1);
}

// 1/x and 1/sqrt(x) from the hardware's seeds, each refined by two Newton
// steps (y' = y (2 - x y) and y' = y (3/2 - x y^2 / 2)): accurate to a few
// units in the last place, not correctly rounded, and much shorter than the
// division and square-root sequences.  x > 0, finite and normal.
__device__ __forceinline__ double rcp_newton(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// Jacobi rotation of the pair with squared norms al, be and product ga:
// false when the pair is orthogonal to working accuracy (ga^2 <= 1e-30 al be).
// t = tan(theta) makes the rotated pair orthogonal: the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga), written without zeta as
// t = 2 ga sgn(be - al) / (|be - al| + sqrt((be - al)^2 + 4 ga^2)), so its
// chain has one square root and one reciprocal; c = 1/sqrt(1 + t^2), s = c t.
// The squared norms become al - t ga and be + t ga.
__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double& c, double& sn, double& t) {
  if (!(ga * ga > 1e-30 * (al * be))) return false;
  const double d = be - al;
  const double r = sqrt(fma(d, d, 4.0 * ga * ga));  // >= 2 |ga| > 0
  t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) * rcp_newton(fabs(d) + r);
  c = rsqrt_newton(fma(t, t, 1.0));  // 1 + t^2 in [1, 2]
  sn = c * t;
  return true;
}

// SVD of a w x w block M (w <= 64, ld) by one-sided Jacobi (Hestenes): the
// columns of M are rotated in pairs until they are mutually orthogonal,
// M Vs = Us diag(sigma); the same rotations accumulate Vs.  Pairs follow a
// round-robin tournament (32 disjoint pairs per round, 63 rounds per sweep;
// columns beyond w are zero and never rotated with another); a pair is rotated
// when (a_p . a_q)^2 > 1e-30 |a_p|^2 |a_q|^2, with tan(theta) from
// zeta = (|a_q|^2 - |a_p|^2) / (2 a_p . a_q).  Sweeps stop when no pair was
// rotated (at most 40).  Then sigma_j = |a_j|, sorted decreasing (ties by
// index), Us[:, j] = a_j / sigma_j (0 when sigma_j = 0).  One workgroup of 1024
// threads: each of the 16 wavefronts takes 2 pairs of a round, lane = row.
constexpr int kSvdThreads = 1024;
__global__ __launch_bounds__(kSvdThreads) void k_utv_svd(int w, const double* __restrict__ M, int64_t ld,
                                                 double* __restrict__ sigma, double* __restrict__ Us,
                                                 double* __restrict__ Vs, int* __restrict__ sweeps_out) {
  constexpr int B = kUtvB;
  __shared__ double sA[B][B + 1];  // [column][row]
  __shared__ double sV[B][B + 1];
  __shared__ double s_norm[B];
  __shared__ double s_n2[B];  // squared column norms, exact at each sweep's start
  __shared__ int s_perm[B];
  __shared__ int s_rot;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < B * B; e += kSvdThreads) {
    const int r = e % B, c = e / B;
    sA[c][r] = (r < w && c < w) ? M[r + (int64_t)c * ld] : 0.0;
    sV[c][r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < kUtvMaxSweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
#pragma unroll
    for (int u = 0; u < B / 16; ++u) {  // 16 wavefronts, 4 columns each
      const int col = wave * (B / 16) + u;
      const double x = sA[col][lane];
      const double n2 = wave_sum(x * x);
      if (lane == 0) s_n2[col] = n2;
    }
    __syncthreads();
    for (int round = 0; round < B - 1; ++round) {
      // the wavefront's two pairs of this round (disjoint: every column is in
      // one pair of a round), all their columns read before any is written
      int p[2], q[2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int k = wave * 2 + kk;
        if (k == 0) {
          p[kk] = round;
          q[kk] = B - 1;
        } else {
          p[kk] = (round + k) % (B - 1);
          q[kk] = (round - k + (B - 1)) % (B - 1);
        }
        if (p[kk] > q[kk]) {
          const int t = p[kk];
          p[kk] = q[kk];
          q[kk] = t;
        }
      }
      double ap[2], aq[2], vp[2], vq[2], al[2], be[2], ga[2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        ap[kk] = sA[p[kk]][lane];
        aq[kk] = sA[q[kk]][lane];
        vp[kk] = sV[p[kk]][lane];
        vq[kk] = sV[q[kk]][lane];
        al[kk] = s_n2[p[kk]];
        be[kk] = s_n2[q[kk]];
      }
      wave_sum2(ap[0] * aq[0], ap[1] * aq[1], lane, ga[0], ga[1]);
      // both pairs' rotations in one pass over the lanes (even lanes: the
      // first pair, odd lanes: the second), then read back as scalars
      const int sel = lane & 1;
      double cl = 1.0, sl = 0.0, tl = 0.0;
      const bool rl = jacobi_rotation(sel ? al[1] : al[0], sel ? be[1] : be[0], sel ? ga[1] : ga[0], cl, sl, tl);
      double c[2], sn[2], t[2];
      bool rot[2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        rot[kk] = __builtin_amdgcn_readlane((int)rl, kk) != 0;
        c[kk] = readlane_d(cl, kk);
        sn[kk] = readlane_d(sl, kk);
        t[kk] = readlane_d(tl, kk);
      }
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        if (!rot[kk]) continue;
        sA[p[kk]][lane] = c[kk] * ap[kk] - sn[kk] * aq[kk];
        sA[q[kk]][lane] = sn[kk] * ap[kk] + c[kk] * aq[kk];
        sV[p[kk]][lane] = c[kk] * vp[kk] - sn[kk] * vq[kk];
        sV[q[kk]][lane] = sn[kk] * vp[kk] + c[kk] * vq[kk];
        if (lane == 0) {
          s_n2[p[kk]] = al[kk] - t[kk] * ga[kk];
          s_n2[q[kk]] = be[kk] + t[kk] * ga[kk];
        }
      }
      if ((rot[0] || rot[1]) && lane == 0) s_rot = 1;
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }
  if (tid < B) {
    double t = 0.0;
    for (int r = 0; r < B; ++r) t += sA[tid][r] * sA[tid][r];
    s_norm[tid] = sqrt(t);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < B; ++j) s_perm[j] = j;
    for (int j = 0; j < w; ++j) {  // selection by decreasing norm, lowest index on ties
      int best = j;
      for (int l = j + 1; l < w; ++l)
        if (s_norm[s_perm[l]] > s_norm[s_perm[best]]) best = l;
      const int t = s_perm[j];
      s_perm[j] = s_perm[best];
      s_perm[best] = t;
    }
    if (sweeps_out) *sweeps_out = sweep;
  }
  __syncthreads();
  for (int e = tid; e < B * B; e += kSvdThreads) {
    const int r = e % B, j = e / B;
    const int c = s_perm[j];
    const double sg = s_norm[c];
    Us[r + j * B] = (j < w && r < w && sg > 0.0) ? sA[c][r] / sg : 0.0;
    Vs[r + j * B] = (j < w && r < w) ? sV[c][r] : 0.0;
    if (r == 0 && j < w) sigma[j] = sg;
  }
}

inline unsigned grid_for(int64_t count) {
  const int64_t g = (count + 255) / 256;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

// Workspace of randUTV (beyond the QR path's): Y and P (n x 64), Z (64 x n),
// the right-application products (n x 128 twice, 128 x n), T's positive form
// (128 x 128), the SVD outputs and the block-product staging (n x 64).
struct UtvWs {
  double* buf = nullptr;
  size_t bytes = 0;
  hipStream_t side = nullptr;  // each step's SVD and the products that use it
  hipStream_t uv = nullptr;    // the products of U and V with the Householder factors
  hipEvent_t pre = nullptr;    // main stream: the step's diagonal block is final
  hipEvent_t done = nullptr;   // side stream: the step's block row and column are final
  hipEvent_t snap[2] = {nullptr, nullptr};     // main stream: a copy set of the factors is written
  hipEvent_t uv_done[2] = {nullptr, nullptr};  // uv stream: a copy set has been used
  hipEvent_t tail = nullptr;                   // side stream: the step's U and V columns are final
};

namespace {

struct UtvBufs {
  double *Y, *P, *Z, *XV, *M, *Vt, *Tp, *sig, *Us, *Vs, *NUsT, *tmp, *tau, *NY;
  int* sweeps;
  // the uv stream's copies of a step's two compact WY forms (V: r x 64,
  // T: 128 x 128, V^T: 64 x r), by step parity, and its XV, M (n x 64)
  double *SVa[2], *STa[2], *SVta[2], *SVu[2], *STu[2], *SVtu[2], *SXV, *SM;
};

hipError_t ensure_utv(lupp_handle_t h, int64_t n, UtvBufs* b) {
  const int64_t B = kUtvB;
  const size_t need = sizeof(double) * (size_t)(2 * n * B + B * n + 2 * n * 128 + 128 * n + 128 * 128 + B +
                                                4 * B * B + n * B + 128 + 64 + 2 * (4 * n * B + 2 * 128 * 128) +
                                                2 * n * B);
  if (!h->utv) {
    h->utv = new (std::nothrow) UtvWs();
    if (!h->utv) return hipErrorOutOfMemory;
  }
  if (need > h->utv->bytes) {
    LUPP_TRY(hipStreamSynchronize(h->stream));
    if (h->utv->buf) (void)hipFree(h->utv->buf);
    h->utv->buf = nullptr;
    h->utv->bytes = 0;
    void* p = nullptr;
    LUPP_TRY(hipMalloc(&p, need));
    h->utv->buf = (double*)p;
    h->utv->bytes = need;
  }
  double* x = h->utv->buf;
  b->Y = x;
  x += n * B;
  b->P = x;
  x += n * B;
  b->Z = x;
  x += B * n;
  b->XV = x;
  x += n * 128;
  b->M = x;
  x += n * 128;
  b->Vt = x;
  x += 128 * n;
  b->Tp = x;
  x += 128 * 128;
  b->sig = x;
  x += B;
  b->Us = x;
  x += B * B;
  b->Vs = x;
  x += B * B;
  b->NUsT = x;
  x += B * B;
  b->NY = x;
  x += B * B;
  b->tmp = x;
  x += n * B;
  b->tau = x;
  x += 128;
  b->sweeps = (int*)x;
  x += 64;
  for (int p = 0; p < 2; ++p) {
    b->SVa[p] = x;
    x += n * B;
    b->SVta[p] = x;
    x += n * B;
    b->SVu[p] = x;
    x += n * B;
    b->SVtu[p] = x;
    x += n * B;
    b->STa[p] = x;
    x += 128 * 128;
    b->STu[p] = x;
    x += 128 * 128;
  }
  b->SXV = x;
  x += n * B;
  b->SM = x;
  UtvWs* w = h->utv;
  if (!w->side) {
    LUPP_TRY(hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking));
    LUPP_TRY(hipStreamCreateWithFlags(&w->uv, hipStreamNonBlocking));
    LUPP_TRY(hipEventCreateWithFlags(&w->pre, hipEventDisableTiming));
    LUPP_TRY(hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
    LUPP_TRY(hipEventCreateWithFlags(&w->tail, hipEventDisableTiming));
    for (int p = 0; p < 2; ++p) {
      LUPP_TRY(hipEventCreateWithFlags(&w->snap[p], hipEventDisableTiming));
      LUPP_TRY(hipEventCreateWithFlags(&w->uv_done[p], hipEventDisableTiming));
    }
  }
  return hipSuccess;
}

// T = -(-T^T)^T and V^T of the compact WY form left by qr_outer (V: r x kb
// at qr_v, ld r; -T^T at qr_tneg, ld 128) into Tp (128 x 128) and Vt (kb x r).
hipError_t prepare_wy(lupp_handle_t h, hipStream_t s, int64_t r, int kb, double* Tp, double* Vt) {
  hipLaunchKernelGGL(k_utv_transpose, dim3(4, 4), dim3(256), 0, s, (int64_t)128, (int64_t)128, qr_tneg(h),
                     (int64_t)128, Tp, (int64_t)128, -1.0);
  hipLaunchKernelGGL(k_utv_transpose, dim3((unsigned)((r + 31) / 32), (unsigned)((kb + 31) / 32)), dim3(256), 0, s, r,
                     (int64_t)kb, qr_v(h), r, Vt, (int64_t)kb, 1.0);
  return hipGetLastError();
}

// X (rows x r, ldx) := X Q with Q = I - V T V^T (V: r x kb, ld r; T: Tp,
// ld 128; V^T: Vt, ld kb), kb = 64 or 128, on stream s: X V, then (X V) T,
// then X -= ((X V) T) V^T (XV and M: rows x kb each).
hipError_t right_apply(hipStream_t s, const double* V, const double* Tp, const double* Vt, double* XV, double* M,
                       int64_t rows, int64_t r, double* X, int64_t ldx, int kb) {
  hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(rows * kb)), dim3(256), 0, s, rows, (int64_t)kb, XV, rows, 0.0);
  hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(rows * kb)), dim3(256), 0, s, rows, (int64_t)kb, M, rows, 0.0);
  LUPP_TRY(hipGetLastError());
  LUPP_TRY(gemm_sub<double>(s, rows, kb, r, X, ldx, V, r, XV, rows, nullptr, 2));      // XV = -X V
  LUPP_TRY(gemm_sub<double>(s, rows, kb, kb, XV, rows, Tp, 128, M, rows, nullptr, 2));  // M = X V T
  LUPP_TRY(gemm_sub<double>(s, rows, r, kb, M, rows, Vt, kb, X, ldx, nullptr, 2));     // X -= M V^T
  return hipSuccess;
}

}  // namespace

void free_utv(lupp_handle_t h) {
  if (!h->utv) return;
  UtvWs* w = h->utv;
  for (hipStream_t st : {w->side, w->uv})
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  for (hipEvent_t e : {w->pre, w->done, w->tail, w->snap[0], w->snap[1], w->uv_done[0], w->uv_done[1]})
    if (e) (void)hipEventDestroy(e);
  if (h->utv->buf) (void)hipFree(h->utv->buf);
  delete h->utv;
  h->utv = nullptr;
}

// A (n x n) := T; U, V (n x n) formed when non-null; G: n x n Gaussian draws.
hipError_t randutv(lupp_handle_t h, int64_t n, double* A, int64_t lda, int q, const double* G, int64_t ldg,
                   double* U, int64_t ldu, double* V, int64_t ldv) {
  constexpr int64_t B = kUtvB;
  hipStream_t s = h->stream;
  LUPP_TRY(ensure_qr(h, n, n));
  UtvBufs b;
  LUPP_TRY(ensure_utv(h, n, &b));
  double* part = qr_part(h);
  auto identity = [&](double* X, int64_t ld) -> hipError_t {
    hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(n * n)), dim3(256), 0, s, n, n, X, ld, 0.0);
    hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(n)), dim3(256), 0, s, (int64_t)1, n, X, ld + 1, 1.0);
    return hipGetLastError();
  };
  if (U) LUPP_TRY(identity(U, ldu));
  if (V) LUPP_TRY(identity(V, ldv));
  // Each step's SVD and the products that use it run on the side stream, so
  // that they overlap the next step's sketch and QR: they write only the
  // step's diagonal block, block row (rows k0 .. k0+w of the columns to the
  // right), block column above it and columns k0 .. of U and V, which the
  // next step does not touch before its right-application to T (it waits
  // there).  The step's products of U and V with its two orthogonal factors
  // also run there, from copies of their compact WY forms (SVa .. SVtu) that
  // the main stream writes after that wait.  The side stream's other buffers
  // (sig, Us, Vs, NUsT, NY, tmp) are its own; XV and M are shared, used by
  // the main stream only before the step's hand-off and after the wait.
  hipStream_t ss = h->utv->side, su = h->utv->uv;
  UtvWs* uw = h->utv;
  bool side_pending = false;
  int uv_last = -1;         // parity of the uv stream's last recorded step, -1 before any
  bool uv_used[2] = {false, false};
  int step = 0;
  // X (rows x w) := X Y (Y w x w, ld 64) through the GEMM: tmp = 0 - X (-Y)
  auto times = [&](double* X, int64_t ldx, int64_t rows, int w, const double* Ysmall) -> hipError_t {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(B * B)), dim3(256), 0, ss, B, B, Ysmall, B, b.NY, B, -1.0);
    hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(rows * w)), dim3(256), 0, ss, rows, (int64_t)w, b.tmp, rows, 0.0);
    LUPP_TRY(hipGetLastError());
    LUPP_TRY(gemm_sub<double>(ss, rows, w, w, X, ldx, b.NY, B, b.tmp, rows, nullptr, 2));
    hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(rows * w)), dim3(256), 0, ss, rows, (int64_t)w, b.tmp, rows, X,
                       ldx, 1.0);
    return hipGetLastError();
  };
  for (int64_t k0 = 0; k0 < n; k0 += B) {
    const int64_t nr = n - k0;
    double* T22 = A + k0 + k0 * lda;
    int w = (int)B;
    if (nr > B) {
      // ---- V_alpha: the sketch Y = (T22^T T22)^q T22^T G_i, nr x 64
      LUPP_TRY(qr_tn(s, nr, nr, G + k0 + k0 * ldg, ldg, T22, lda, 64, part, b.Z));  // Z = G_i^T T22
      hipLaunchKernelGGL(k_utv_transpose, dim3(2, (unsigned)((nr + 31) / 32)), dim3(256), 0, s, B, nr, b.Z, B, b.Y,
                         nr, 1.0);
      LUPP_TRY(hipGetLastError());
      for (int it = 0; it < q; ++it) {
        hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(nr * B)), dim3(256), 0, s, nr, B, b.P, nr, 0.0);
        LUPP_TRY(hipGetLastError());
        LUPP_TRY(gemm_sub<double>(s, nr, B, nr, T22, lda, b.Y, nr, b.P, nr, nullptr, 2));  // P = -T22 Y
        LUPP_TRY(qr_tn(s, nr, nr, b.P, nr, T22, lda, 64, part, b.Z));                     // Z = P^T T22
        hipLaunchKernelGGL(k_utv_transpose, dim3(2, (unsigned)((nr + 31) / 32)), dim3(256), 0, s, B, nr, b.Z, B, b.Y,
                           nr, -1.0);  // Y = -Z^T = T22^T T22 Y
        LUPP_TRY(hipGetLastError());
      }
      // Householder QR of Y; T[:, k0:] and V[:, k0:] times its Q (after the
      // previous step's block row is final)
      LUPP_TRY(qr_outer(h, nr, B, b.Y, nr, b.tau, B, true));
      if (side_pending) LUPP_TRY(hipStreamWaitEvent(s, h->utv->done, 0));
      LUPP_TRY(prepare_wy(h, s, nr, 64, b.Tp, b.Vt));
      LUPP_TRY(right_apply(s, qr_v(h), b.Tp, b.Vt, b.XV, b.M, n, nr, A + k0 * lda, lda, 64));
      const int par = step & 1;
      // the copy set of this parity was last read by the uv stream two steps ago
      if ((U || V) && uv_used[par]) LUPP_TRY(hipStreamWaitEvent(s, uw->uv_done[par], 0));
      if (V) {  // V[:, k0:] times this Q on the uv stream: copy the form
        hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(nr * B)), dim3(256), 0, s, nr, B, qr_v(h), nr,
                           b.SVa[par], nr, 1.0);
        hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(128 * 128)), dim3(256), 0, s, (int64_t)128, (int64_t)128,
                           b.Tp, (int64_t)128, b.STa[par], (int64_t)128, 1.0);
        hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(nr * B)), dim3(256), 0, s, B, nr, b.Vt, B, b.SVta[par], B,
                           1.0);
        LUPP_TRY(hipGetLastError());
      }
      // ---- U_alpha: Householder QR of T22's first 64 columns, applied to
      // the rest of T22; U[:, k0:] times its Q (side stream, from a copy of
      // its form); the block column below the diagonal (the reflectors) becomes 0
      LUPP_TRY(qr_outer(h, nr, nr, T22, lda, b.tau, B, true));
      if (U) {
        LUPP_TRY(prepare_wy(h, s, nr, 64, b.STu[par], b.SVtu[par]));
        hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(nr * B)), dim3(256), 0, s, nr, B, qr_v(h), nr,
                           b.SVu[par], nr, 1.0);
        LUPP_TRY(hipGetLastError());
      }
      hipLaunchKernelGGL(k_utv_zero_lower, dim3(grid_for(nr * B)), dim3(256), 0, s, nr, (int)B, T22, lda);
      LUPP_TRY(hipGetLastError());
      if (U || V) {  // the uv stream: V[:, k0:] and U[:, k0:] times the step's two factors
        LUPP_TRY(hipEventRecord(uw->snap[par], s));
        LUPP_TRY(hipStreamWaitEvent(su, uw->snap[par], 0));
        if (V) LUPP_TRY(right_apply(su, b.SVa[par], b.STa[par], b.SVta[par], b.SXV, b.SM, n, nr, V + k0 * ldv, ldv, 64));
        if (U) LUPP_TRY(right_apply(su, b.SVu[par], b.STu[par], b.SVtu[par], b.SXV, b.SM, n, nr, U + k0 * ldu, ldu, 64));
        LUPP_TRY(hipEventRecord(uw->uv_done[par], su));
        uv_used[par] = true;
        uv_last = par;
      }
    } else {
      w = (int)nr;
    }
    // ---- U_beta, V_beta: SVD of the w x w diagonal block (side stream),
    // after the step's products of V and U with its two Householder factors
    LUPP_TRY(hipEventRecord(h->utv->pre, s));
    LUPP_TRY(hipStreamWaitEvent(ss, h->utv->pre, 0));

    hipLaunchKernelGGL(k_utv_svd, dim3(1), dim3(kSvdThreads), 0, ss, w, T22, lda, b.sig, b.Us, b.Vs, b.sweeps);
    hipLaunchKernelGGL(k_utv_transpose, dim3(2, 2), dim3(256), 0, ss, B, B, b.Us, B, b.NUsT, B, -1.0);  // -Us^T
    hipLaunchKernelGGL(k_utv_set_diag, dim3(1), dim3(256), 0, ss, w, b.sig, T22, lda);
    LUPP_TRY(hipGetLastError());
    const int64_t nright = n - k0 - w;
    if (nright > 0) {  // T[k0:k0+w, k0+w:] := Us^T T[k0:k0+w, k0+w:]
      double* X = T22 + w * lda;
      hipLaunchKernelGGL(k_utv_fill, dim3(grid_for(w * nright)), dim3(256), 0, ss, (int64_t)w, nright, b.tmp, B,
                         0.0);
      LUPP_TRY(hipGetLastError());
      LUPP_TRY(gemm_sub<double>(ss, w, nright, w, b.NUsT, B, X, lda, b.tmp, B, nullptr, 2));  // tmp = Us^T X
      hipLaunchKernelGGL(k_utv_scale_copy, dim3(grid_for(w * nright)), dim3(256), 0, ss, (int64_t)w, nright, b.tmp,
                         B, X, lda, 1.0);
      LUPP_TRY(hipGetLastError());
    }
    LUPP_TRY(times(A + k0 * lda, lda, k0, w, b.Vs));       // T[:k0, k0:k0+w] := T[:k0, k0:k0+w] Vs
    LUPP_TRY(hipEventRecord(uw->done, ss));
    side_pending = true;
    if (U || V) {  // after the uv stream's products over these columns
      if (uv_last >= 0) LUPP_TRY(hipStreamWaitEvent(ss, uw->uv_done[uv_last], 0));
      if (U) LUPP_TRY(times(U + k0 * ldu, ldu, n, w, b.Us));  // U[:, k0:k0+w] := U[:, k0:k0+w] Us
      if (V) LUPP_TRY(times(V + k0 * ldv, ldv, n, w, b.Vs));  // V[:, k0:k0+w] := V[:, k0:k0+w] Vs
      LUPP_TRY(hipEventRecord(uw->tail, ss));
    }
    ++step;
  }
  // the caller's stream carries the end of the factorization
  if (side_pending) LUPP_TRY(hipStreamWaitEvent(s, uw->done, 0));
  if ((U || V) && side_pending) LUPP_TRY(hipStreamWaitEvent(s, uw->tail, 0));
  if (uv_last >= 0) LUPP_TRY(hipStreamWaitEvent(s, uw->uv_done[uv_last], 0));
  return hipSuccess;
}

}  // namespace lupp

extern "C" int lupp_drandutv(lupp_handle_t h, int64_t n, double* dA, int64_t lda, int32_t q, const double* dG,
                             int64_t ldg, double* dU, int64_t ldu, double* dV, int64_t ldv) {
  if (!h) return -1;
  if (n < 0 || n > 131072) return -2;
  if (!dA && n > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (q < 0 || q > 16) return -5;
  if (!dG && n > 0) return -6;
  if (ldg < (n > 1 ? n : 1)) return -7;
  if (dU && ldu < (n > 1 ? n : 1)) return -9;
  if (dV && ldv < (n > 1 ? n : 1)) return -11;
  if (n == 0) return LUPP_OK;
  const hipError_t e = lupp::randutv(h, n, dA, lda, q, dG, ldg, dU, ldu, dV, ldv);
  return e == hipErrorOutOfMemory ? LUPP_ERR_ALLOC : lupp::hip_status(e);
}
