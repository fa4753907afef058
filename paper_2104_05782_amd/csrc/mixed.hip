// lupp_dgesv_mixed: FP32 factorization with low-precision trailing updates,
// then FP64 iterative refinement against the original FP64 matrix, classical
// (Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed., Ch. 12)
// or GMRES-based (Carson and Higham, SIAM J. Sci. Comput. 40, 2018).  All
// vector work runs in the library's kernels on the handle's stream; the host
// keeps only scalars: the stopping tests, and the small Hessenberg
// least-squares problem of GMRES (Givens rotations, back substitution).
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "handle.h"

namespace lupp {

namespace {
constexpr int64_t kResidualChunks = 16;  // column chunks of the deterministic residual
constexpr int kMaxRestart = 60;          // Arnoldi basis <= 61 vectors (mdot handles <= 64)
}  // namespace

struct MixedWs {
  int64_t n = 0, m = 0;  // capacity: order and GMRES restart length
  void* base = nullptr;  // one allocation holding everything below
  float* A32 = nullptr;  // n x n, lda = n: the FP32 copy, then its factors
  int32_t* ipiv = nullptr;
  int32_t* info = nullptr;
  int32_t* perm = nullptr;  // row permutation composed from ipiv: (P v)[i] = v[perm[i]]
  double* x = nullptr;      // iterate
  double* xbest = nullptr;  // iterate with the smallest backward error so far
  double* r = nullptr;      // residual
  double* t = nullptr;      // temporary
  double* d = nullptr;      // correction
  double* zero = nullptr;   // zeros (right-hand side of t = -A v)
  float* z32 = nullptr;     // FP32 right-hand side of the triangular solves
  double* part = nullptr;   // partial sums of the residual and dot products
  double* V = nullptr;      // Arnoldi basis, n x (m + 1)
  double* hdev = nullptr;   // 3 x 64: projections of both passes and the norm
  unsigned long long* mx = nullptr;  // max-abs slots (bit patterns of doubles)
};

void free_mixed(lupp_handle_t h) {
  if (!h->mixed) return;
  if (h->mixed->base) (void)hipFree(h->mixed->base);
  delete h->mixed;
  h->mixed = nullptr;
}

namespace {

// Layout of the mixed solve's single allocation for order n and restart m.
struct MixedLayout {
  size_t oA, oi, ov, oz, op, oV, oh, total;
};
MixedLayout mixed_layout(int64_t n, int64_t m) {
  const int64_t nblk = (n + 255) / 256;
  int64_t part = kResidualChunks * n;
  if (nblk * 64 > part) part = nblk * 64;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  MixedLayout L;
  size_t off = 0;
  L.oA = off;
  off += al((size_t)n * n * 4);
  L.oi = off;
  off += al((size_t)n * 4 * 2 + 64);  // ipiv, perm, info
  L.ov = off;
  off += al((size_t)n * 8) * 6;  // x, xbest, r, t, d, zero
  L.oz = off;
  off += al((size_t)n * 4);
  L.op = off;
  off += al((size_t)part * 8);
  L.oV = off;
  off += al((size_t)n * (m + 1) * 8);
  L.oh = off;
  off += al(3 * 64 * 8 + 16 * 8);
  L.total = off;
  return L;
}

hipError_t ensure_mixed(lupp_handle_t h, int64_t n, int64_t m) {
  MixedWs* w = h->mixed;
  if (w && w->n >= n && w->m >= m) return hipSuccess;
  LUPP_TRY(hipStreamSynchronize(h->stream));
  if (w && w->n > n) n = w->n;
  if (w && w->m > m) m = w->m;
  free_mixed(h);
  w = new (std::nothrow) MixedWs();
  if (!w) return hipErrorOutOfMemory;
  const MixedLayout Lo = mixed_layout(n, m);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, Lo.total);
  if (e != hipSuccess) {
    delete w;
    return e;
  }
  char* b = (char*)p;
  w->base = p;
  w->n = n;
  w->m = m;
  w->A32 = (float*)(b + Lo.oA);
  w->ipiv = (int32_t*)(b + Lo.oi);
  w->perm = w->ipiv + n;
  w->info = w->perm + n;
  double* vs = (double*)(b + Lo.ov);
  const size_t vstride = al((size_t)n * 8) / 8;
  w->x = vs;
  w->xbest = vs + vstride;
  w->r = vs + 2 * vstride;
  w->t = vs + 3 * vstride;
  w->d = vs + 4 * vstride;
  w->zero = vs + 5 * vstride;
  w->z32 = (float*)(b + Lo.oz);
  w->part = (double*)(b + Lo.op);
  w->V = (double*)(b + Lo.oV);
  w->hdev = (double*)(b + Lo.oh);
  w->mx = (unsigned long long*)(w->hdev + 3 * 64);
  h->mixed = w;
  LUPP_TRY(hipMemsetAsync(w->zero, 0, (size_t)n * 8, h->stream));
  return hipSuccess;
}

inline double bits_to_double(unsigned long long u) {
  double v;
  memcpy(&v, &u, sizeof v);
  return v;
}

struct Ctx {
  lupp_handle_t h;
  MixedWs* w;
  hipStream_t s;
  int64_t n;
  const double* A;
  int64_t lda;
  double anorm = 0.0;
};

// out = sign * inv(U) inv(L) P v with the FP32 factors (v scaled by its
// max-norm for the FP32 solve; mx slot `slot` holds that norm).
hipError_t precond(Ctx& c, const double* v, double sign, double* out, int slot) {
  MixedWs* w = c.w;
  LUPP_TRY(hipMemsetAsync(w->mx + slot, 0, sizeof(unsigned long long), c.s));
  LUPP_TRY(absmax(c.s, c.n, v, w->mx + slot));
  LUPP_TRY(gather_scale(c.s, c.n, w->perm, v, w->mx + slot, w->z32));
  LUPP_TRY(trsv_wave<float>(c.s, true, c.n, w->A32, c.n, w->z32, &c.h->trsv));
  LUPP_TRY(trsv_wave<float>(c.s, false, c.n, w->A32, c.n, w->z32, &c.h->trsv));
  return axpy_dev(c.s, c.n, sign, w->mx + slot, w->z32, nullptr, out);
}

// r = b - A x and the backward error eta(x) = ||r||inf / (||A||inf ||x||inf + ||b||inf)
hipError_t backward_error(Ctx& c, const double* x, const double* b, double bnorm, double* eta) {
  MixedWs* w = c.w;
  LUPP_TRY(residual(c.s, c.n, c.A, c.lda, x, b, w->r, w->part, kResidualChunks));
  LUPP_TRY(hipMemsetAsync(w->mx, 0, 2 * sizeof(unsigned long long), c.s));
  LUPP_TRY(absmax(c.s, c.n, w->r, w->mx));
  LUPP_TRY(absmax(c.s, c.n, x, w->mx + 1));
  unsigned long long hm[2];
  LUPP_TRY(hipMemcpyAsync(hm, w->mx, sizeof hm, hipMemcpyDeviceToHost, c.s));
  LUPP_TRY(hipStreamSynchronize(c.s));
  const double rn = bits_to_double(hm[0]), xn = bits_to_double(hm[1]);
  const double den = c.anorm * xn + bnorm;
  *eta = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
  return hipSuccess;
}

// One GMRES cycle on inv(M) A d = inv(M) r (M = P^T L U in FP32), d from 0:
// at most m Arnoldi steps, stopped when the estimated preconditioned residual
// falls to inner_tol times its initial value.
hipError_t gmres_cycle(Ctx& c, int m, double inner_tol, int* steps) {
  MixedWs* w = c.w;
  const int64_t n = c.n;
  double* V = w->V;
  *steps = 0;
  LUPP_TRY(precond(c, w->r, 1.0, V, 2));
  LUPP_TRY(mdot(c.s, n, 1, V, n, V, w->part, w->hdev));
  double beta2 = 0.0;
  LUPP_TRY(hipMemcpyAsync(&beta2, w->hdev, sizeof beta2, hipMemcpyDeviceToHost, c.s));
  LUPP_TRY(hipStreamSynchronize(c.s));
  const double beta = std::sqrt(beta2);
  if (!(beta > 0.0) || !std::isfinite(beta)) return hipMemsetAsync(w->d, 0, (size_t)n * 8, c.s);
  LUPP_TRY(scale_copy(c.s, n, 1.0 / beta, V, V));
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
  g[0] = beta;
  int k = 0;
  std::vector<double> hh(3 * 64);
  for (int j = 0; j < m; ++j) {
    double* vj = V + (int64_t)j * n;
    double* wv = V + (int64_t)(j + 1) * n;
    // wv = inv(M) A vj, through t = 0 - A vj and a negated preconditioner
    LUPP_TRY(residual(c.s, n, c.A, c.lda, vj, w->zero, w->t, w->part, kResidualChunks));
    LUPP_TRY(precond(c, w->t, -1.0, wv, 2));
    // classical Gram-Schmidt, twice
    LUPP_TRY(mdot(c.s, n, j + 1, V, n, wv, w->part, w->hdev));
    LUPP_TRY(mgemv_sub(c.s, n, j + 1, V, n, w->hdev, wv));
    LUPP_TRY(mdot(c.s, n, j + 1, V, n, wv, w->part, w->hdev + 64));
    LUPP_TRY(mgemv_sub(c.s, n, j + 1, V, n, w->hdev + 64, wv));
    LUPP_TRY(mdot(c.s, n, 1, wv, n, wv, w->part, w->hdev + 128));
    LUPP_TRY(hipMemcpyAsync(hh.data(), w->hdev, hh.size() * 8, hipMemcpyDeviceToHost, c.s));
    LUPP_TRY(hipStreamSynchronize(c.s));
    for (int i = 0; i <= j; ++i) Hij(i, j) = hh[i] + hh[64 + i];
    const double hn = std::sqrt(hh[128]);
    Hij(j + 1, j) = hn;
    // previous rotations, then a new one that zeroes H(j+1, j)
    for (int i = 0; i < j; ++i) {
      const double a = Hij(i, j), bb = Hij(i + 1, j);
      Hij(i, j) = cs[i] * a + sn[i] * bb;
      Hij(i + 1, j) = -sn[i] * a + cs[i] * bb;
    }
    const double a = Hij(j, j), bb = Hij(j + 1, j);
    const double rr = std::hypot(a, bb);
    if (rr > 0.0) {
      cs[j] = a / rr;
      sn[j] = bb / rr;
    } else {
      cs[j] = 1.0;
      sn[j] = 0.0;
    }
    Hij(j, j) = rr;
    Hij(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    k = j + 1;
    if (!(hn > 0.0) || !std::isfinite(hn)) break;  // breakdown: the Krylov space is invariant
    if (std::fabs(g[j + 1]) <= inner_tol * beta) break;
    if (j + 1 < m) LUPP_TRY(scale_copy(c.s, n, 1.0 / hn, wv, wv));
  }
  *steps = k;
  // y = H(0:k, 0:k) \ g(0:k), d = V(:, 0:k) y
  std::vector<double> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double sacc = g[i];
    for (int q = i + 1; q < k; ++q) sacc -= Hij(i, q) * y[q];
    y[i] = Hij(i, i) != 0.0 ? sacc / Hij(i, i) : 0.0;
  }
  LUPP_TRY(hipMemcpyAsync(w->hdev, y.data(), (size_t)k * 8, hipMemcpyHostToDevice, c.s));
  LUPP_TRY(hipMemsetAsync(w->d, 0, (size_t)n * 8, c.s));
  LUPP_TRY(mgemv_add(c.s, n, k, V, n, w->hdev, w->d));
  return hipStreamSynchronize(c.s);  // y lives on the host stack
}

// FP64 factorization and solve of one right-hand side on a fresh copy of A.
hipError_t fallback_fp64(Ctx& c, const double* b, double bnorm, double* x_out, double* eta) {
  const int64_t n = c.n;
  void* p = nullptr;
  LUPP_TRY(hipMalloc(&p, (size_t)n * n * 8 + (size_t)n * 4 + 256));
  double* Ad = (double*)p;
  int32_t* ipiv = (int32_t*)(Ad + (size_t)n * n);
  int32_t* info = ipiv + n;
  hipError_t e = hipMemcpy2DAsync(Ad, (size_t)n * 8, c.A, (size_t)c.lda * 8, (size_t)n * 8, (size_t)n,
                                  hipMemcpyDeviceToDevice, c.s);
  if (e == hipSuccess) e = getrf<double>(c.h, n, n, Ad, n, ipiv, info);
  if (e == hipSuccess) e = hipMemcpyAsync(c.w->t, b, (size_t)n * 8, hipMemcpyDeviceToDevice, c.s);
  if (e == hipSuccess) e = getrs<double>(c.h, n, 1, Ad, n, ipiv, c.w->t, n);
  if (e == hipSuccess) e = backward_error(c, c.w->t, b, bnorm, eta);
  if (e == hipSuccess) e = hipMemcpyAsync(x_out, c.w->t, (size_t)n * 8, hipMemcpyDeviceToDevice, c.s);
  if (e == hipSuccess) e = hipStreamSynchronize(c.s);
  (void)hipFree(p);
  return e;
}

int rank_status(int st) {
  // severity order for the aggregate over right-hand sides
  switch (st) {
    case LUPP_IR_CONVERGED: return 0;
    case LUPP_IR_STAGNATED: return 1;
    case LUPP_IR_MAXITER: return 2;
    case LUPP_IR_DIVERGED: return 3;
    default: return 4;
  }
}

int gesv_mixed(lupp_handle_t h, int64_t n, int64_t nrhs, const double* A, int64_t lda, const double* B,
               int64_t ldb, double* X, int64_t ldx, const lupp_ir_opts& o, lupp_ir_report& rep) {
  using clk = std::chrono::steady_clock;
  hipStream_t s = h->stream;
  const int m = o.solver == LUPP_IR_GMRES ? o.gmres_restart : 1;
  hipError_t e = ensure_workspace(h);
  if (e == hipSuccess) e = ensure_mixed(h, n, m);
  if (e == hipSuccess) e = ensure_trsv(h, n);
  if (e == hipSuccess && o.factor_prec != LUPP_PREC_FP32) e = ensure_lp_scale(h, n, n, o.nb > 0 ? o.nb : h->nb);
  if (e != hipSuccess) return LUPP_ERR_ALLOC;
  MixedWs* w = h->mixed;
  Ctx c{h, w, s, n, A, lda};

  // factorization of the FP32 copy
  const auto t0 = clk::now();
  const int64_t nb_saved = h->nb;
  const int prec_saved = h->update_prec;
  if (o.nb > 0) h->nb = o.nb;
  h->update_prec = o.factor_prec;
  e = d2s_mat(s, n, n, A, lda, w->A32, n);
  if (e == hipSuccess) e = getrf<float>(h, n, n, w->A32, n, w->ipiv, w->info);
  h->nb = nb_saved;
  h->update_prec = prec_saved;
  std::vector<int32_t> ipiv(n), perm(n);
  int32_t info = 0;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && h->side) e = hipStreamSynchronize(h->side);
  if (e == hipSuccess && h->bulk) e = hipStreamSynchronize(h->bulk);
  if (e == hipSuccess) e = hipMemcpy(ipiv.data(), w->ipiv, (size_t)n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&info, w->info, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e);
  int32_t werr = 0;
  if (hipMemcpy(&werr, &h->slots->err, 4, hipMemcpyDeviceToHost) == hipSuccess && werr) return LUPP_ERR_INTERNAL;
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t q = ipiv[k] - 1;
    if (q < k || q >= n) return LUPP_ERR_INTERNAL;
    const int32_t tmp = perm[k];
    perm[k] = perm[q];
    perm[q] = tmp;
  }
  e = hipMemcpy(w->perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_status(e);
  rep.info = info;
  rep.factor_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();

  const auto t1 = clk::now();
  rep.status = LUPP_IR_CONVERGED;
  rep.iters = 0;
  rep.inner_iters = 0;
  rep.fallback_used = 0;
  rep.backward_error = 0.0;
  {
    e = hipMemsetAsync(w->mx + 2, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) e = norm_inf_mat(s, n, A, lda, w->part, kResidualChunks, w->mx + 2);
    unsigned long long an = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&an, w->mx + 2, sizeof an, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e);
    c.anorm = bits_to_double(an);
  }
  for (int64_t j = 0; j < nrhs; ++j) {
    const double* b = B + j * ldb;
    double* xo = X + j * ldx;
    unsigned long long bn = 0;
    e = hipMemsetAsync(w->mx + 3, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) e = absmax(s, n, b, w->mx + 3);
    if (e == hipSuccess) e = hipMemcpyAsync(&bn, w->mx + 3, sizeof bn, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemsetAsync(w->x, 0, (size_t)n * 8, s);
    if (e != hipSuccess) return hip_status(e);
    const double bnorm = bits_to_double(bn);
    int status = LUPP_IR_MAXITER, iters = 0;
    double eta = 0.0, best = INFINITY;
    std::vector<double> hist;
    if (info > 0) status = LUPP_IR_SINGULAR;
    while (info == 0) {
      e = backward_error(c, w->x, b, bnorm, &eta);
      if (e != hipSuccess) return hip_status(e);
      hist.push_back(eta);
      if (eta <= o.tol) {
        status = LUPP_IR_CONVERGED;
        best = eta;
        e = hipMemcpyAsync(w->xbest, w->x, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        break;
      }
      if (!std::isfinite(eta) || eta > 10.0 * best) {
        status = LUPP_IR_DIVERGED;
        break;
      }
      if (eta < best) {
        best = eta;
        e = hipMemcpyAsync(w->xbest, w->x, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_status(e);
      }
      const size_t q = hist.size();
      if (q >= 3 && hist[q - 1] > 0.5 * hist[q - 3]) {
        status = LUPP_IR_STAGNATED;
        break;
      }
      if (iters >= o.max_iter) {
        status = LUPP_IR_MAXITER;
        break;
      }
      if (o.solver == LUPP_IR_GMRES) {
        int steps = 0;
        e = gmres_cycle(c, m, o.inner_tol, &steps);
        rep.inner_iters += steps;
      } else {
        e = precond(c, w->r, 1.0, w->d, 2);
      }
      if (e == hipSuccess) e = vec_add(s, n, w->d, w->x);
      if (e != hipSuccess) return hip_status(e);
      ++iters;
    }
    if (status != LUPP_IR_SINGULAR) {
      eta = best;
      e = hipMemcpyAsync(xo, w->xbest, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_status(e);
    } else {
      eta = INFINITY;
      e = hipMemsetAsync(xo, 0, (size_t)n * 8, s);
      if (e != hipSuccess) return hip_status(e);
    }
    if (status != LUPP_IR_CONVERGED && o.fallback_fp64) {
      double eta64 = INFINITY;
      e = fallback_fp64(c, b, bnorm, xo, &eta64);
      if (e != hipSuccess) return hip_status(e);
      eta = eta64;
      rep.fallback_used += 1;
    }
    if (rank_status(status) > rank_status(rep.status)) rep.status = status;
    if (iters > rep.iters) rep.iters = iters;
    if (!(eta <= rep.backward_error)) rep.backward_error = eta;
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_status(e);
  if (take_trsv_error(h) != 0) return LUPP_ERR_INTERNAL;
  rep.refine_ms = std::chrono::duration<double, std::milli>(clk::now() - t1).count();
  return LUPP_OK;
}

}  // namespace

size_t mixed_workspace_bytes(int64_t n, int64_t restart) { return mixed_layout(n, restart).total; }

}  // namespace lupp

extern "C" {

void lupp_ir_opts_default(lupp_ir_opts* o, int32_t solver) {
  if (!o) return;
  o->factor_prec = LUPP_PREC_FP16;
  o->solver = solver == LUPP_IR_CLASSICAL ? LUPP_IR_CLASSICAL : LUPP_IR_GMRES;
  o->tol = 1e-14;
  o->max_iter = o->solver == LUPP_IR_GMRES ? 10 : 50;
  o->gmres_restart = 30;
  o->inner_tol = 1e-6;
  o->nb = 0;
  o->fallback_fp64 = 0;
}

int lupp_dgesv_mixed(lupp_handle_t h, int64_t n, int64_t nrhs, const double* dA, int64_t lda, const double* dB,
                     int64_t ldb, double* dX, int64_t ldx, const lupp_ir_opts* opts, lupp_ir_report* rep) {
  if (!h) return -1;
  if (n < 0 || n > (int64_t)lupp::kLeafMaxGroups * 1024) return -2;
  if (nrhs < 0) return -3;
  if (!dA && n > 0) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (!dB && n > 0 && nrhs > 0) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  if (!dX && n > 0 && nrhs > 0) return -8;
  if (ldx < (n > 1 ? n : 1)) return -9;
  lupp_ir_opts o;
  if (opts) o = *opts;
  else lupp_ir_opts_default(&o, LUPP_IR_GMRES);
  if (o.factor_prec < LUPP_PREC_FP32 || o.factor_prec > LUPP_PREC_FP8_E4M3) return -10;
  if (o.solver != LUPP_IR_CLASSICAL && o.solver != LUPP_IR_GMRES) return -10;
  if (!(o.tol > 0.0) || o.max_iter < 1 || o.max_iter > 1000) return -10;
  if (o.solver == LUPP_IR_GMRES && (o.gmres_restart < 1 || o.gmres_restart > lupp::kMaxRestart)) return -10;
  if (o.solver == LUPP_IR_GMRES && !(o.inner_tol > 0.0 && o.inner_tol < 1.0)) return -10;
  if (o.nb < 0 || o.nb > 1024) return -10;
  lupp_ir_report r{};
  int rc = LUPP_OK;
  if (n > 0 && nrhs > 0) rc = lupp::gesv_mixed(h, n, nrhs, dA, lda, dB, ldb, dX, ldx, o, r);
  if (rep) *rep = r;
  return rc;
}

}  // extern "C"
