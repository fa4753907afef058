// C ABI and host-side drivers of the blocked right-looking LU with partial
// pivoting (declarations and conventions: include/lupp.h).
//
// The loop is the paper's FLAME loop (Section 4.3: partition A into
// A_TL, A_TR, A_BL, A_BR with A_TL empty; while A_TL does not cover A,
// repartition with a b x b block A11, b = min(nb, n(A_BR)); update; continue
// with the boundaries moved past A11), instantiated for LU:
//   [A11; A21], p1 := LUPP([A11; A21])        column block (recursive)
//   apply p1 to [A10; A20] and [A12; A22]      laswp
//   A12 := inv(L11) * A12                       trsm (recursive, GEMM inside)
//   A22 := A22 - A21 * A12                      GEMM on MFMA
// Loop invariant after a step with A_TL of order k: the top k rows and left k
// columns hold L_TL\U_TL, U_TR and L_BL of P_k*A, and A_BR holds its Schur
// complement P_k*A_BR - L_BL*U_TR.
#include <stdio.h>
#include <stdlib.h>

#include <new>
#include <type_traits>
#include <vector>

#include <algorithm>

#include "handle.h"

namespace lupp {

// Phase timing: HIP events on the handle's stream around a phase's launches
// (level 1: every phase; level 2: the trailing updates only).
int timer_begin(lupp_handle_t h, int phase, hipStream_t st) {
  if (h->timing == 0 || (h->timing == 2 && phase != LUPP_PHASE_UPDATE)) return -1;
  if (h->nrecords == h->records.size()) {
    TimingRecord r;
    if (hipEventCreate(&r.start) != hipSuccess) return -1;
    if (hipEventCreate(&r.stop) != hipSuccess) {
      (void)hipEventDestroy(r.start);
      return -1;
    }
    h->records.push_back(r);
  }
  TimingRecord& r = h->records[h->nrecords];
  if (hipEventRecord(r.start, st) != hipSuccess) return -1;
  r.phase = phase;
  r.big = false;
  r.flops = 0.0;
  r.bytes = 0.0;
  return (int)h->nrecords++;
}

void timer_end(lupp_handle_t h, int idx, hipStream_t st, double flops, bool big, double bytes) {
  if (idx < 0) return;
  TimingRecord& r = h->records[idx];
  r.flops = flops;
  r.bytes = bytes;
  r.big = big;
  (void)hipEventRecord(r.stop, st);
}

namespace {

constexpr int kLookaheadPanelCUs = 32;
constexpr int kLookaheadPanelCUs2 = 64;  // second pair, for panels of 33 to 64 workgroups

// Epoch of the panel kernel's progress flags: every launch uses flag values
// above all values written before; the flags are cleared before wrap-around.
inline hipError_t next_epoch(lupp_handle_t h, hipStream_t st, int w, uint32_t* out) {
  if (h->epoch > 0xF0000000u) {
    LUPP_TRY(reset_flags(st, h->slots));
    h->epoch = 0;
  }
  *out = h->epoch;
  h->epoch += (uint32_t)w + 1u;
  return hipSuccess;
}

// Algorithmic bytes of an update C (M x N) -= A (M x K) * B (K x N): C read
// and written once, A and B read once.
template <typename T>
double update_bytes(int64_t M, int64_t N, int64_t K) {
  return (double)sizeof(T) * (2.0 * (double)M * (double)N + ((double)M + (double)N) * (double)K);
}

// B (w x ncols) := inv(L) * B with L unit lower triangular (w x w).
template <typename T>
hipError_t trsm_lower_unit(hipStream_t s, int64_t w, int64_t ncols, const T* L, int64_t ldl, T* B, int64_t ldb) {
  if (w <= kTrsmBandMaxW) return trsm_lower_band<T>(s, w, ncols, L, ldl, B, ldb);
  const int64_t w1 = w / 2;
  LUPP_TRY(trsm_lower_unit<T>(s, w1, ncols, L, ldl, B, ldb));
  LUPP_TRY(gemm_sub<T>(s, w - w1, ncols, w1, L + w1, ldl, B, ldb, B + w1, ldb));
  return trsm_lower_unit<T>(s, w - w1, ncols, L + w1 + w1 * ldl, ldl, B + w1, ldb);
}

// B (w x ncols) := inv(U) * B with U upper triangular, non-unit (w x w).
template <typename T>
hipError_t trsm_upper(hipStream_t s, int64_t w, int64_t ncols, const T* U, int64_t ldu, T* B, int64_t ldb) {
  if (w <= 64) return trsm_small<T>(s, false, w, ncols, U, ldu, B, ldb);
  const int64_t w1 = w / 2;
  LUPP_TRY(trsm_upper<T>(s, w - w1, ncols, U + w1 + w1 * ldu, ldu, B + w1, ldb));
  LUPP_TRY(gemm_sub<T>(s, w1, ncols, w - w1, U + w1 * ldu, ldu, B + w1, ldb, B, ldb));
  return trsm_upper<T>(s, w1, ncols, U, ldu, B, ldb);
}

// Column-block factorization of columns [k, k+w), rows [k, m), inside the
// enclosing column block [p0, p1): blocks up to h->block columns wide are one
// cooperative launch that also applies its interchanges to every other column
// of [p0, p1); wider blocks split in two (left half; U12 := inv(L11) * A12;
// A22 -= A21 * U12; right half, which also interchanges rows of the left).
template <typename T>
hipError_t panel(lupp_handle_t h, hipStream_t s, int64_t m, int64_t k, int64_t w, int64_t p0, int64_t p1, T* A,
                 int64_t lda, int32_t* ipiv, int32_t* info) {
  if (w <= h->block) {
    uint32_t ep;
    LUPP_TRY(next_epoch(h, s, (int)block_tags((int)w), &ep));
    const int t = timer_begin(h, LUPP_PHASE_PANEL_LEAF, s);
    LUPP_TRY(panel_block<T>(s, m - k, (int)w, A + k + k * lda, lda, ipiv, k, info, h->slots, ep, p0 - k, p1 - k));
    timer_end(h, t, s, 0.0);
    return hipSuccess;
  }
  int64_t w1 = w / 2;
  if (w1 > 16) w1 = (w1 / 16) * 16;
  const int64_t w2 = w - w1;
  LUPP_TRY(panel<T>(h, s, m, k, w1, p0, p1, A, lda, ipiv, info));
  int t = timer_begin(h, LUPP_PHASE_PANEL_TRSM, s);
  LUPP_TRY(trsm_lower_unit<T>(s, w1, w2, A + k + k * lda, lda, A + k + (k + w1) * lda, lda));
  timer_end(h, t, s, (double)w1 * (double)w1 * (double)w2);
  t = timer_begin(h, LUPP_PHASE_PANEL_GEMM, s);
  LUPP_TRY(gemm_sub<T>(s, m - k - w1, w2, w1, A + (k + w1) + k * lda, lda, A + k + (k + w1) * lda, lda,
                       A + (k + w1) + (k + w1) * lda, lda));
  timer_end(h, t, s, 2.0 * (double)(m - k - w1) * (double)w2 * (double)w1);
  return panel<T>(h, s, m, k + w1, w2, p0, p1, A, lda, ipiv, info);
}

// Trailing update C -= A * B of the outer loop: FP64 and FP32 on the MFMA GEMM
// of the working precision, or (FP32 factorization with a low-precision update
// format) on the low-precision GEMM; `which` selects the low-precision
// workspace slot of the updates that may run concurrently (0: next block,
// 1: bulk, 2: the bulk's share on the panel's CUs or the dataflow runtime's
// first lookahead stream, 3: its second).
template <typename T>
hipError_t update(lupp_handle_t h, hipStream_t s, int which, int64_t M, int64_t N, int64_t K, const T* A,
                  int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc, int* tile = nullptr) {
  if constexpr (std::is_same<T, float>::value) {
    if (h->update_prec != LUPP_PREC_FP32) {
      if (tile) *tile = 1;
      return gemm_lp_sub(s, h->update_prec, M, N, K, A, lda, B, ldb, C, ldc, h->lp_scale[which],
                         h->lp_packed ? h->lp_pack[which] : nullptr, h->lp_pack_cap);
    }
  }
  return gemm_sub<T>(s, M, N, K, A, lda, B, ldb, C, ldc, tile, which == 2 ? 1 : 0);
}

// Reads the panel and bulk-update times of an earlier step once its events
// have completed (never waits), and keeps running estimates.
void harvest_split_timings(lupp_handle_t h) {
  for (int o = 0; o < 2; ++o) {
    if (!h->tm_pending[o]) continue;
    const hipError_t q1 = hipEventQuery(h->tm_ev[o][1]);
    const hipError_t q3 = hipEventQuery(h->tm_ev[o][3]);
    (void)hipGetLastError();  // a not-ready query is not an error of the factorization
    if (q1 != hipSuccess || q3 != hipSuccess) continue;
    float pm = 0.f, bm = 0.f;
    if (hipEventElapsedTime(&pm, h->tm_ev[o][0], h->tm_ev[o][1]) == hipSuccess &&
        hipEventElapsedTime(&bm, h->tm_ev[o][2], h->tm_ev[o][3]) == hipSuccess && bm > 0.f) {
      const int pr = h->tm_pair[o];
      h->est_panel_ms[pr] = h->est_panel_ms[pr] < 0 ? pm : 0.5 * (h->est_panel_ms[pr] + pm);
      const int pcus = pr == 0 ? h->panel_cus : h->panel_cus2;
      const double rate = h->tm_flops[o] / ((double)bm * (double)(h->ncu - pcus));
      h->est_rate = h->est_rate < 0 ? rate : 0.5 * (h->est_rate + rate);
    }
    (void)hipGetLastError();
    h->tm_pending[o] = false;
  }
}

// Columns of the remaining-columns update (nc columns, M x nc x K) to run on
// the panel's CUs after the panel, so that both shares end together: with
// bulk CUs B, panel CUs S, panel time P and per-CU rate R, the bulk share f
// of the W flops solves f W / (B R) = P + (1 - f) W / (S R).  Zero when the
// panel alone outlasts the whole update.
int64_t side_columns(lupp_handle_t h, int pair, int64_t M, int64_t nc, int64_t K, bool fp64) {
  const int pcus = pair == 0 ? h->panel_cus : h->panel_cus2;
  const double B = (double)(h->ncu - pcus), S = (double)pcus;
  if (B <= 0 || S <= 0) return 0;
  const double P =
      h->est_panel_ms[pair] >= 0 ? h->est_panel_ms[pair] : (fp64 ? 2.3 : 1.8) * (pair + 1) * (double)K / 256.0;
  double R = h->est_rate;
  if (R <= 0) R = fp64 ? 2.0e8 : (h->update_prec != LUPP_PREC_FP32 ? 6.0e8 : 3.0e8);
  const double W = 2.0 * (double)M * (double)nc * (double)K;
  if (W / (B * R) <= P) return 0;
  const double f = (P * R + W / S) / (W * (1.0 / B + 1.0 / S));
  int64_t ns = (int64_t)((1.0 - f) * (double)nc);
  ns = (ns / 128) * 128;
  if (ns < 256 || ns > nc - 128) return 0;
  return ns;
}

// Column block [k, k+b): factor it on stream st, with its phase timing.
template <typename T>
hipError_t factor_block(lupp_handle_t h, hipStream_t st, int64_t m, int64_t k, int64_t b, T* A, int64_t lda,
                        int32_t* ipiv, int32_t* info) {
  const int t = timer_begin(h, LUPP_PHASE_PANEL, st);
  LUPP_TRY(panel<T>(h, st, m, k, b, k, k + b, A, lda, ipiv, info));
  timer_end(h, t, st, 0.0);
  return hipSuccess;
}

}  // namespace

// Blocked right-looking factorization with depth-1 lookahead: while the bulk
// of step k's trailing update runs on the main stream, the next column block
// (whose columns are updated first) is factored on the side stream.  The
// paper removes the same synchronization point of the column-block
// factorization by scheduling its tasks out of order (Section 4.1,
// algorithm-by-blocks; Section 4.4, the runtime's dataflow order); here the
// dataflow is fixed and expressed with two streams and two events per step.
template <typename T>
hipError_t getrf_dag(lupp_handle_t h, int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* info,
                     int depth);

template <typename T>
hipError_t getrf(lupp_handle_t h, int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* info) {
  hipStream_t s = h->stream;
  const int64_t p = m < n ? m : n;
  // lookahead deeper than one step: the dataflow runtime (needs the lookahead
  // streams and the deferred interchanges of the finished columns)
  if (h->lookahead >= 2 && p > 0 && h->side && h->bulk && ensure_look_streams(h) && h->look &&
      ensure_defer(h, m, n, sizeof(T)))
    return getrf_dag<T>(h, m, n, A, lda, ipiv, info, h->lookahead);
  LUPP_TRY(set_int(s, info, 0));
  if (p == 0) return hipSuccess;
  const bool la = h->lookahead && h->side && h->bulk;
  const int64_t J = (p + h->nb - 1) / h->nb;
  const bool defer = ensure_defer(h, m, n, sizeof(T));
  SwapPairs* step_pairs = defer ? (SwapPairs*)h->defer_buf : nullptr;
  LUPP_TRY(factor_block<T>(h, s, m, 0, (p < h->nb) ? p : h->nb, A, lda, ipiv, info));
  for (int64_t k = 0; k < p; k += h->nb) {
    const int64_t b = (p - k < h->nb) ? (p - k) : h->nb;
    const int64_t kn = k + b;
    const int64_t bn = (kn < p) ? ((p - kn < h->nb) ? (p - kn) : h->nb) : 0;
    const int64_t nr = n - kn;                    // columns right of the block
    const int64_t mr = m - kn;                    // rows below it
    const int64_t n1 = (nr > 0 && mr > 0) ? bn : 0;  // the next block's columns
    // The block's interchanges, composed once into pairs, go to the next
    // block's columns here, to the other columns on the right together with
    // their update below, and to the finished columns on the left either now
    // or (deferred) once at the end.
    const bool composed = b <= kMaxSwaps;
    SwapPairs* sp = defer ? step_pairs + k / h->nb : h->pairs;
    int t = timer_begin(h, LUPP_PHASE_LASWP, s);
    if (composed) {
      LUPP_TRY(swap_pairs(s, ipiv, k, kn, m, sp));
      if (!defer) LUPP_TRY(apply_pairs<T>(s, A, lda, 0, k, 0, 0, sp, 2 * b));
      LUPP_TRY(apply_pairs<T>(s, A, lda, kn, kn + n1, 0, 0, sp, 2 * b));
    } else {
      LUPP_TRY(laswp<T>(s, A, lda, m, 0, n, k, kn, ipiv, k, kn, nullptr));
    }
    timer_end(h, t, s, 0.0);
    if (nr <= 0) continue;
    if (n1 > 0) {
      t = timer_begin(h, LUPP_PHASE_TRSM, s);
      LUPP_TRY(trsm_lower_unit<T>(s, b, n1, A + k + k * lda, lda, A + k + kn * lda, lda));
      timer_end(h, t, s, (double)b * (double)b * (double)n1);
      // columns of the next block first, so that it can be factored early
      int tile = -1;
      t = timer_begin(h, LUPP_PHASE_UPDATE, s);
      LUPP_TRY(update<T>(h, s, 0, mr, n1, b, A + kn + k * lda, lda, A + k + kn * lda, lda, A + kn + kn * lda, lda,
                         &tile));
      timer_end(h, t, s, 2.0 * (double)mr * (double)n1 * (double)b, tile == 1, update_bytes<T>(mr, n1, b));
    }
    // overlap only when the next block's cooperative factorization fits in
    // the reserved CUs (one workgroup per CU at most)
    // a pair of streams whose panel CUs hold the next block's cooperative
    // factorization (one workgroup per CU at most)
    const int G = panel_groups(mr);
    const int pair = (G <= h->panel_cus) ? 0 : (h->side2 && h->bulk2 && G <= h->panel_cus2) ? 1 : -1;
    const bool overlap = la && n1 > 0 && pair >= 0 && nr > n1;
    hipStream_t sside = pair == 1 ? h->side2 : h->side, sbulk = pair == 1 ? h->bulk2 : h->bulk;
    hipStream_t su = s;
    int slot = -1;  // timing slot of this step's panel and bulk update, if measured
    if (overlap) {
      LUPP_TRY(hipEventRecord(h->ev_cols, s));
      LUPP_TRY(hipStreamWaitEvent(sside, h->ev_cols, 0));
      LUPP_TRY(hipStreamWaitEvent(sbulk, h->ev_cols, 0));
      if (h->split) {
        harvest_split_timings(h);
        if (!h->tm_pending[h->tm_slot]) slot = h->tm_slot;
      }
      if (slot >= 0) LUPP_TRY(hipEventRecord(h->tm_ev[slot][0], sside));
      LUPP_TRY(factor_block<T>(h, sside, m, kn, bn, A, lda, ipiv, info));
      if (slot >= 0) LUPP_TRY(hipEventRecord(h->tm_ev[slot][1], sside));
      su = sbulk;
    }
    if (nr > n1) {
      const int64_t c1 = kn + n1, nc = nr - n1;
      if (composed) {
        t = timer_begin(h, LUPP_PHASE_LASWP, su);
        LUPP_TRY(apply_pairs<T>(su, A, lda, c1, n, 0, 0, sp, 2 * b));
        timer_end(h, t, su, 0.0);
      }
      t = timer_begin(h, LUPP_PHASE_TRSM, su);
      LUPP_TRY(trsm_lower_unit<T>(su, b, nc, A + k + k * lda, lda, A + k + c1 * lda, lda));
      timer_end(h, t, su, (double)b * (double)b * (double)nc);
      if (mr > 0) {
        // the bulk CUs take the first columns; once the next block is
        // factored, the panel's CUs take the last ones
        const int64_t nside = (overlap && h->split) ? side_columns(h, pair, mr, nc, b, sizeof(T) == 8) : 0;
        const int64_t nbulk = nc - nside;
        if (nside > 0) {
          LUPP_TRY(hipEventRecord(h->ev_trsm, su));
          LUPP_TRY(hipStreamWaitEvent(sside, h->ev_trsm, 0));
        }
        int tile = -1;
        if (slot >= 0) LUPP_TRY(hipEventRecord(h->tm_ev[slot][2], su));
        t = timer_begin(h, LUPP_PHASE_UPDATE, su);
        LUPP_TRY(update<T>(h, su, 1, mr, nbulk, b, A + kn + k * lda, lda, A + k + c1 * lda, lda, A + kn + c1 * lda,
                           lda, &tile));
        timer_end(h, t, su, 2.0 * (double)mr * (double)nbulk * (double)b, tile == 1, update_bytes<T>(mr, nbulk, b));
        if (slot >= 0) {
          LUPP_TRY(hipEventRecord(h->tm_ev[slot][3], su));
          h->tm_flops[slot] = 2.0 * (double)mr * (double)nbulk * (double)b;
          h->tm_pair[slot] = pair;
          h->tm_pending[slot] = true;
          h->tm_slot ^= 1;
        }
        if (nside > 0) {
          const int64_t c2 = c1 + nbulk;
          t = timer_begin(h, LUPP_PHASE_UPDATE, sside);
          LUPP_TRY(update<T>(h, sside, 2, mr, nside, b, A + kn + k * lda, lda, A + k + c2 * lda, lda,
                             A + kn + c2 * lda, lda));
          timer_end(h, t, sside, 2.0 * (double)mr * (double)nside * (double)b, false, update_bytes<T>(mr, nside, b));
        }
      }
    }
    if (overlap) {
      LUPP_TRY(hipEventRecord(h->ev_panel, sside));
      LUPP_TRY(hipEventRecord(h->ev_bulk, sbulk));
      LUPP_TRY(hipStreamWaitEvent(s, h->ev_bulk, 0));
      LUPP_TRY(hipStreamWaitEvent(s, h->ev_panel, 0));
    } else if (n1 > 0) {
      LUPP_TRY(factor_block<T>(h, s, m, kn, bn, A, lda, ipiv, info));
    }
  }
  if (defer && J >= 2) {
    // every later step's interchanges on the finished blocks, one pass
    const int t = timer_begin(h, LUPP_PHASE_LASWP, s);
    int32_t* g = (int32_t*)((char*)h->defer_buf + (size_t)J * sizeof(SwapPairs));
    int32_t* gmap = g + 2 * m;
    LUPP_TRY(left_maps(s, step_pairs, J, m, h->nb, g, gmap));
    LUPP_TRY(left_gather<T>(s, A, lda, m, h->nb, J, gmap));
    timer_end(h, t, s, 0.0);
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- algorithm-by-blocks
// The dataflow form of the same factorization: the paper's algorithm-by-
// blocks (Section 4.1) with its runtime's two parts (Section 4.4, the
// analyzer and the dispatcher).  The blocked loop is unrolled into tasks on
// operands, the analyzer derives each task's predecessors from the operands
// it reads and writes (read after write, write after read, write after
// write), and the dispatcher issues the tasks in a priority order onto HIP
// streams, turning each dependency on a task of another stream into an event
// wait, so that the GPU runs every task as soon as its inputs are final.
//
// Operands: column block j of width nb (object j, rows from the block's
// step down) and the interchange record of step k (object J + k).  Tasks:
//   START        zeroes info; writes every object (everything follows it);
//   PANEL(k)     factors column block k and composes its interchanges into
//                the step's record; writes k and J + k;
//   UPD(k, a, b) the record's interchanges, U := inv(L11) U and the update
//                A22 -= L21 U on the columns of blocks a .. b-1 right of the
//                factored block; reads k and J + k, writes a .. b-1 (a = k
//                only for the tail of a last factored block narrower than nb);
//   LEFT         the deferred interchanges of the finished blocks; reads
//                J .. 2J-1, writes 0 .. J-2.
// With lookahead depth d, step k's update of block k+1 and of blocks
// k+2 .. k+d are tasks of their own, the rest one task (one large update), so
// the chain of column blocks may run up to d steps ahead of the large
// updates.  Streams: the column blocks on a CU-masked panel stream; the next
// block's update on the caller's stream (nothing else runs then on the
// panel's CUs: the next column block waits for it); the other lookahead
// blocks' updates and the large updates on two streams masked to the CUs
// outside the panel's, so that they never slow the column block down.  Partial pivoting is
// unchanged: every column block spans the full remaining height, and each
// task computes exactly what the same step computes in the loop above, in
// the same order per entry (the factors are identical bit for bit).
struct DagTask {
  int kind;             // 0 start, 1 panel, 2 update, 3 left interchanges
  int64_t k, a, b;      // step; column blocks [a, b)
  hipStream_t stream;
  std::vector<int> reads, writes, deps;
};

// Analyzer: predecessors of every task from its read and write sets.
void dag_analyze(std::vector<DagTask>& t, int nobj) {
  std::vector<int> last_writer(nobj, -1);
  std::vector<std::vector<int>> readers(nobj);
  for (int i = 0; i < (int)t.size(); ++i) {
    std::vector<int>& d = t[i].deps;
    for (int o : t[i].reads)
      if (last_writer[o] >= 0) d.push_back(last_writer[o]);  // read after write
    for (int o : t[i].writes) {
      if (last_writer[o] >= 0) d.push_back(last_writer[o]);  // write after write
      for (int r : readers[o]) d.push_back(r);               // write after read
    }
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    d.erase(std::remove(d.begin(), d.end(), i), d.end());
    for (int o : t[i].reads) readers[o].push_back(i);
    for (int o : t[i].writes) {
      last_writer[o] = i;
      readers[o].clear();
    }
  }
}

hipError_t dag_events(lupp_handle_t h, size_t count) {
  while (h->dag_events.size() < count) {
    hipEvent_t e = nullptr;
    LUPP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->dag_events.push_back(e);
  }
  return hipSuccess;
}

template <typename T>
hipError_t getrf_dag(lupp_handle_t h, int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* info,
                     int depth) {
  hipStream_t s = h->stream;
  const int64_t p = m < n ? m : n;
  const int64_t nb = h->nb;
  const int64_t J = (p + nb - 1) / nb;   // column blocks that are factored
  const int64_t JN = (n + nb - 1) / nb;  // column blocks of the matrix
  const int NOBJ = (int)(JN + J);
  SwapPairs* step_pairs = (SwapPairs*)h->defer_buf;
  // the panel stream of step k (rows left: m - k nb), or null when its
  // cooperative factorization exceeds the reserved CUs (it then runs on the
  // caller's stream)
  auto pair_of = [&](int64_t k) {
    const int G = panel_groups(m - k * nb);
    return (G <= h->panel_cus) ? 0 : (h->side2 && h->bulk2 && h->look2 && G <= h->panel_cus2) ? 1 : -1;
  };
  std::vector<DagTask> t;
  auto add = [&](int kind, int64_t k, int64_t a, int64_t b, hipStream_t st) -> DagTask& {
    t.push_back(DagTask{kind, k, a, b, st, {}, {}, {}});
    return t.back();
  };
  {
    DagTask& st = add(0, 0, 0, 0, s);
    for (int o = 0; o < NOBJ; ++o) st.writes.push_back(o);
  }
  for (int64_t k = 0; k < J; ++k) {
    const int pr = pair_of(k);
    DagTask& pt = add(1, k, k, k + 1, pr == 0 ? h->side : pr == 1 ? h->side2 : s);
    pt.writes = {(int)k, (int)(JN + k)};
    // the columns right of the factored block: [k nb + b, n), from object a0
    // on (a0 = k when the last factored block is narrower than nb)
    const int64_t kn = k * nb + ((p - k * nb < nb) ? (p - k * nb) : nb);
    if (kn >= n) continue;
    const int64_t a0 = kn / nb;
    // the large update runs beside the next step's column block: the bulk
    // stream whose CUs are disjoint from that block's panel stream
    const int prn = (k + 1 < J) ? pair_of(k + 1) : 0;
    hipStream_t sb = prn == 1 ? h->bulk2 : h->bulk;
    hipStream_t sl = prn == 1 ? h->look2 : h->look;
    const int64_t la = a0 + depth < JN ? a0 + depth : JN;  // end of the lookahead blocks
    const int64_t cut[4] = {a0, a0 + 1 < la ? a0 + 1 : la, la, JN};
    for (int q = 0; q < 3; ++q) {
      if (cut[q] >= cut[q + 1]) continue;
      DagTask& u = add(2, k, cut[q], cut[q + 1], q == 0 ? s : q == 1 ? sl : sb);
      u.reads = {(int)k, (int)(JN + k)};
      for (int64_t j = cut[q]; j < cut[q + 1]; ++j) u.writes.push_back((int)j);
    }
  }
  if (J >= 2) {
    DagTask& lt = add(3, 0, 0, 0, s);
    for (int64_t k = 0; k < J; ++k) lt.reads.push_back((int)(JN + k));
    for (int64_t j = 0; j < J - 1; ++j) lt.writes.push_back((int)j);
  }
  dag_analyze(t, NOBJ);
  LUPP_TRY(dag_events(h, t.size()));

  // Dispatcher: list order is the priority (each step's column block, then
  // the update of the next block, the lookahead blocks, the large update).
  for (size_t i = 0; i < t.size(); ++i) {
    const DagTask& x = t[i];
    for (int d : x.deps)
      if (t[d].stream != x.stream) LUPP_TRY(hipStreamWaitEvent(x.stream, h->dag_events[d], 0));
    const int64_t k0 = x.k * nb;
    const int64_t b = (p - k0 < nb) ? (p - k0) : nb;
    if (x.kind == 0) {
      LUPP_TRY(set_int(s, info, 0));
    } else if (x.kind == 1) {
      LUPP_TRY(factor_block<T>(h, x.stream, m, k0, b, A, lda, ipiv, info));
      const int tt = timer_begin(h, LUPP_PHASE_LASWP, x.stream);
      LUPP_TRY(swap_pairs(x.stream, ipiv, k0, k0 + b, m, step_pairs + x.k));
      timer_end(h, tt, x.stream, 0.0);
    } else if (x.kind == 2) {
      const int64_t kn = k0 + b, mr = m - kn;
      const int64_t c0 = (x.a * nb > kn) ? x.a * nb : kn, c1 = (x.b * nb < n) ? x.b * nb : n, nc = c1 - c0;
      const SwapPairs* sp = step_pairs + x.k;
      int tt = timer_begin(h, LUPP_PHASE_LASWP, x.stream);
      LUPP_TRY(apply_pairs<T>(x.stream, A, lda, c0, c1, 0, 0, sp, 2 * b));
      timer_end(h, tt, x.stream, 0.0);
      tt = timer_begin(h, LUPP_PHASE_TRSM, x.stream);
      LUPP_TRY(trsm_lower_unit<T>(x.stream, b, nc, A + k0 + k0 * lda, lda, A + k0 + c0 * lda, lda));
      timer_end(h, tt, x.stream, (double)b * (double)b * (double)nc);
      if (mr > 0) {
        int tile = -1;
        tt = timer_begin(h, LUPP_PHASE_UPDATE, x.stream);
        // one workspace slot per stream: updates on different streams may overlap
        const int slot = x.stream == s ? 0 : (x.stream == h->look ? 2 : (x.stream == h->look2 ? 3 : 1));
        LUPP_TRY(update<T>(h, x.stream, slot, mr, nc, b, A + kn + k0 * lda, lda, A + k0 + c0 * lda, lda,
                           A + kn + c0 * lda, lda, &tile));
        timer_end(h, tt, x.stream, 2.0 * (double)mr * (double)nc * (double)b, tile == 1, update_bytes<T>(mr, nc, b));
      }
    } else {
      const int tt = timer_begin(h, LUPP_PHASE_LASWP, s);
      int32_t* g = (int32_t*)((char*)h->defer_buf + (size_t)J * sizeof(SwapPairs));
      int32_t* gmap = g + 2 * m;
      LUPP_TRY(left_maps(s, step_pairs, J, m, nb, g, gmap));
      LUPP_TRY(left_gather<T>(s, A, lda, m, nb, J, gmap));
      timer_end(h, tt, s, 0.0);
    }
    LUPP_TRY(hipEventRecord(h->dag_events[i], x.stream));
  }
  // the caller's stream ends after every task (LEFT and the last steps'
  // tasks on other streams)
  for (size_t i = 0; i < t.size(); ++i)
    if (t[i].stream != s) LUPP_TRY(hipStreamWaitEvent(s, h->dag_events[i], 0));
  return hipSuccess;
}

// Solve with the factors: the interchanges in runs of at most kMaxSwaps
// (composed per run, applied to all right-hand sides at once), then the two
// triangular solves -- for one or two right-hand sides the one-launch
// wavefront solve (reads each factor once), otherwise the recursive trsm.
template <typename T>
hipError_t getrs(lupp_handle_t h, int64_t n, int64_t nrhs, const T* LU, int64_t lda, const int32_t* ipiv, T* B,
                 int64_t ldb) {
  hipStream_t s = h->stream;
  LUPP_TRY(diag_zero_check<T>(s, n, LU, lda, h->trsv.sing));
  for (int64_t k1 = 0; k1 < n; k1 += kMaxSwaps) {
    const int64_t k2 = (n - k1 < kMaxSwaps) ? n : k1 + kMaxSwaps;
    LUPP_TRY(laswp<T>(s, B, ldb, n, 0, nrhs, 0, 0, ipiv, k1, k2, h->pairs));
  }
  if (nrhs <= 2) {
    for (int64_t j = 0; j < nrhs; ++j) {
      LUPP_TRY(trsv_wave<T>(s, true, n, LU, lda, B + j * ldb, &h->trsv));
      LUPP_TRY(trsv_wave<T>(s, false, n, LU, lda, B + j * ldb, &h->trsv));
    }
    return hipSuccess;
  }
  LUPP_TRY(trsm_lower_unit<T>(s, n, nrhs, LU, lda, B, ldb));
  return trsm_upper<T>(s, n, nrhs, LU, lda, B, ldb);
}

template hipError_t getrf<double>(lupp_handle_t, int64_t, int64_t, double*, int64_t, int32_t*, int32_t*);
template hipError_t getrf<float>(lupp_handle_t, int64_t, int64_t, float*, int64_t, int32_t*, int32_t*);
template hipError_t getrs<double>(lupp_handle_t, int64_t, int64_t, const double*, int64_t, const int32_t*, double*,
                                  int64_t);
template hipError_t getrs<float>(lupp_handle_t, int64_t, int64_t, const float*, int64_t, const int32_t*, float*,
                                 int64_t);

hipError_t ensure_lp_scale(lupp_handle_t h, int64_t m, int64_t n, int64_t nb) {
  const int64_t need = gemm_lp_scale_slots(m, n);
  const size_t pneed = h->lp_packed ? gemm_lp_pack_bytes(m, n, nb) : 0;
  if (need <= h->lp_scale_cap && pneed <= h->lp_pack_cap) return hipSuccess;
  LUPP_TRY(hipStreamSynchronize(h->stream));
  if (h->bulk) LUPP_TRY(hipStreamSynchronize(h->bulk));
  if (h->side) LUPP_TRY(hipStreamSynchronize(h->side));
  if (h->bulk2) LUPP_TRY(hipStreamSynchronize(h->bulk2));
  if (h->look) LUPP_TRY(hipStreamSynchronize(h->look));
  if (h->look2) LUPP_TRY(hipStreamSynchronize(h->look2));
  if (h->side2) LUPP_TRY(hipStreamSynchronize(h->side2));
  const int64_t ns = need > h->lp_scale_cap ? need : h->lp_scale_cap;
  const size_t np = pneed > h->lp_pack_cap ? pneed : h->lp_pack_cap;
  if (h->lp_scale[0]) (void)hipFree(h->lp_scale[0]);
  if (h->lp_pack[0]) (void)hipFree(h->lp_pack[0]);
  for (int i = 0; i < 4; ++i) {
    h->lp_scale[i] = nullptr;
    h->lp_pack[i] = nullptr;
  }
  h->lp_scale_cap = 0;
  h->lp_pack_cap = 0;
  void* p = nullptr;
  LUPP_TRY(hipMalloc(&p, (size_t)ns * 4 * sizeof(int)));
  for (int i = 0; i < 4; ++i) h->lp_scale[i] = (int*)p + i * ns;
  h->lp_scale_cap = ns;
  if (np > 0) {
    const size_t slot = (np + 255) / 256 * 256;
    void* q = nullptr;
    LUPP_TRY(hipMalloc(&q, slot * 4));
    for (int i = 0; i < 4; ++i) h->lp_pack[i] = (char*)q + i * slot;
    h->lp_pack_cap = slot;
  }
  return hipSuccess;
}

hipError_t ensure_trsv(lupp_handle_t h, int64_t n) {
  const int64_t need = (n + 63) / 64;
  TrsvState& t = h->trsv;
  if (need <= t.max_blocks && t.epoch < 0xF0000000u) return hipSuccess;
  LUPP_TRY(hipStreamSynchronize(h->stream));
  if (need > t.max_blocks) {
    if (t.flags) (void)hipFree(t.flags);
    t.flags = nullptr;
    t.max_blocks = 0;
    const int64_t cap = need < 1024 ? 1024 : need;
    void* p = nullptr;
    // flags, then the ticket counter and the error flag
    LUPP_TRY(hipMalloc(&p, (size_t)cap * sizeof(uint32_t) + 64));
    t.flags = (uint32_t*)p;
    t.ticket = (uint64_t*)((char*)p + ((size_t)cap * sizeof(uint32_t) + 7) / 8 * 8);
    t.err = (int32_t*)(t.ticket + 1);
    t.sing = t.err + 1;
    t.max_blocks = cap;
    LUPP_TRY(hipMemsetAsync(p, 0, (size_t)cap * sizeof(uint32_t) + 64, h->stream));
    t.tickets = 0;
  } else {
    LUPP_TRY(hipMemsetAsync(t.flags, 0, (size_t)t.max_blocks * sizeof(uint32_t), h->stream));
  }
  t.epoch = 0;
  return hipSuccess;
}

// The dataflow runtime's lookahead-update streams, masked like the bulk
// streams (created on its first use, so the loop path holds none).
bool ensure_look_streams(lupp_handle_t h) {
  if (h->look) return true;
  const int ncu = h->ncu;
  if (ncu <= 0 || h->panel_cus <= 0) return false;
  std::vector<uint32_t> mb((ncu + 31) / 32, 0u), mb2((ncu + 31) / 32, 0u);
  for (int c = 0; c < ncu; ++c) {
    if (c >= h->panel_cus) mb[c / 32] |= 1u << (c % 32);
    if (c >= kLookaheadPanelCUs2) mb2[c / 32] |= 1u << (c % 32);
  }
  if (hipExtStreamCreateWithCUMask(&h->look, (uint32_t)mb.size(), mb.data()) != hipSuccess) {
    h->look = nullptr;
    return false;
  }
  if (h->panel_cus2 > 0 &&
      hipExtStreamCreateWithCUMask(&h->look2, (uint32_t)mb2.size(), mb2.data()) != hipSuccess)
    h->look2 = nullptr;
  return true;
}

bool ensure_defer(lupp_handle_t h, int64_t m, int64_t n, size_t elem) {
  const int64_t p = m < n ? m : n;
  const int64_t nb = h->nb;
  const int64_t J = (p + nb - 1) / nb;
  if (!h->defer || J < 2 || nb > kMaxSwaps || m - nb > left_gather_max_rows(elem) || (J - 1) * nb > 0x7fffffff)
    return false;
  const size_t bytes = (size_t)J * sizeof(SwapPairs) + sizeof(int32_t) * (size_t)(2 * m + left_map_entries(J, m, nb));
  if (bytes > ((size_t)1 << 30)) return false;
  if (bytes > h->defer_bytes) {
    if (h->defer_buf) {
      if (hipStreamSynchronize(h->stream) != hipSuccess) return false;
      (void)hipFree(h->defer_buf);
      h->defer_buf = nullptr;
      h->defer_bytes = 0;
    }
    if (hipMalloc(&h->defer_buf, bytes) != hipSuccess) {
      h->defer_buf = nullptr;
      return false;
    }
    h->defer_bytes = bytes;
  }
  return true;
}

hipError_t ensure_workspace(lupp_handle_t h) {
  if (h->slots) return hipSuccess;
  void* p = nullptr;
  const size_t bytes = sizeof(LeafSlots) + sizeof(SwapPairs);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e;
  e = hipMemset(p, 0, bytes);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return e;
  }
  h->slots = (LeafSlots*)p;
  h->pairs = (SwapPairs*)((char*)p + sizeof(LeafSlots));
  h->epoch = 0;
  // lookahead streams: the panel's CUs and the bulk update's CUs are disjoint,
  // so the latency-bound panel is not slowed by co-resident GEMM workgroups
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu < 64) {
    h->lookahead = 0;
    return hipSuccess;
  }
  h->panel_cus = kLookaheadPanelCUs;
  std::vector<uint32_t> mside((ncu + 31) / 32, 0u), mbulk((ncu + 31) / 32, 0u);
  for (int c = 0; c < ncu; ++c) {
    if (c < h->panel_cus) mside[c / 32] |= 1u << (c % 32);
    else mbulk[c / 32] |= 1u << (c % 32);
  }
  if (hipExtStreamCreateWithCUMask(&h->side, (uint32_t)mside.size(), mside.data()) != hipSuccess) h->side = nullptr;
  if (hipExtStreamCreateWithCUMask(&h->bulk, (uint32_t)mbulk.size(), mbulk.data()) != hipSuccess) h->bulk = nullptr;
  if (ncu >= 2 * kLookaheadPanelCUs2) {
    std::vector<uint32_t> m2s((ncu + 31) / 32, 0u), m2b((ncu + 31) / 32, 0u);
    for (int c = 0; c < ncu; ++c) {
      if (c < kLookaheadPanelCUs2) m2s[c / 32] |= 1u << (c % 32);
      else m2b[c / 32] |= 1u << (c % 32);
    }
    if (hipExtStreamCreateWithCUMask(&h->side2, (uint32_t)m2s.size(), m2s.data()) != hipSuccess) h->side2 = nullptr;
    if (hipExtStreamCreateWithCUMask(&h->bulk2, (uint32_t)m2b.size(), m2b.data()) != hipSuccess) h->bulk2 = nullptr;
    if (h->side2 && h->bulk2) h->panel_cus2 = kLookaheadPanelCUs2;
  }
  if (!h->side || !h->bulk || hipEventCreateWithFlags(&h->ev_cols, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_bulk, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_trsm, hipEventDisableTiming) != hipSuccess)
    h->lookahead = 0;
  h->ncu = ncu;
  for (int o = 0; o < 2; ++o)
    for (int e = 0; e < 4; ++e)
      if (hipEventCreate(&h->tm_ev[o][e]) != hipSuccess) h->split = 0;
  return hipSuccess;
}

int take_trsv_error(lupp_handle_t h) {
  TrsvState& t = h->trsv;
  if (!t.err) return 0;
  int32_t err = 0;
  if (hipMemcpy(&err, t.err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  if (!err) return 0;
  const int32_t zero = 0;
  uint64_t dev = 0;
  if (hipMemcpy(t.err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(&dev, t.ticket, sizeof(dev), hipMemcpyDeviceToHost) != hipSuccess)
    return -1;
  t.tickets = dev;
  return err;
}

size_t getrf_workspace_bytes(lupp_handle_t h, int64_t m, int64_t n, size_t elem) {
  size_t bytes = sizeof(LeafSlots) + sizeof(SwapPairs);
  const int64_t p = m < n ? m : n;
  const int64_t nb = h->nb;
  const int64_t J = (p + nb - 1) / nb;
  if (h->defer && J >= 2 && nb <= kMaxSwaps && m - nb <= left_gather_max_rows(elem) && (J - 1) * nb <= 0x7fffffff) {
    const size_t d = (size_t)J * sizeof(SwapPairs) + sizeof(int32_t) * (size_t)(2 * m + left_map_entries(J, m, nb));
    if (d <= ((size_t)1 << 30)) bytes += d;
  }
  if (elem == 4 && h->update_prec != LUPP_PREC_FP32) {
    bytes += (size_t)gemm_lp_scale_slots(m, n) * 4 * sizeof(int);
    if (h->lp_packed) bytes += (gemm_lp_pack_bytes(m, n, nb) + 255) / 256 * 256 * 4;
  }
  return bytes;
}

size_t trsv_workspace_bytes(int64_t n) {
  const int64_t need = (n + 63) / 64;
  return (size_t)(need < 1024 ? 1024 : need) * sizeof(uint32_t) + 64;
}

namespace {

template <typename T>
int getrf_entry(lupp_handle_t h, int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* info) {
  if (!h) return -1;
  if (m < 0 || m >= ((int64_t)1 << 31)) return -2;
  if (n < 0) return -3;
  if (!A && m > 0 && n > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (!ipiv && m > 0 && n > 0) return -6;
  if (!info) return -7;
  if (m > (int64_t)kLeafMaxGroups * 1024) return LUPP_ERR_UNSUPPORTED;
  hipError_t e = ensure_workspace(h);
  if (e != hipSuccess) return LUPP_ERR_ALLOC;
  if (std::is_same<T, float>::value && h->update_prec != LUPP_PREC_FP32) {
    e = ensure_lp_scale(h, m, n, h->nb);
    if (e != hipSuccess) return LUPP_ERR_ALLOC;
  }
  return hip_status(getrf<T>(h, m, n, A, lda, ipiv, info));
}

template <typename T>
int getrs_entry(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const T* LU, int64_t lda, const int32_t* ipiv,
                T* B, int64_t ldb) {
  if (!h) return -1;
  if (trans != 'N' && trans != 'n') return -2;
  if (n < 0 || n >= ((int64_t)1 << 31)) return -3;
  if (nrhs < 0) return -4;
  if (!LU && n > 0) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (!ipiv && n > 0) return -7;
  if (!B && n > 0 && nrhs > 0) return -8;
  if (ldb < (n > 1 ? n : 1)) return -9;
  if (n == 0 || nrhs == 0) return LUPP_OK;
  hipError_t e = ensure_workspace(h);
  if (e == hipSuccess) e = ensure_trsv(h, nrhs <= 2 ? n : 1);
  if (e != hipSuccess) return LUPP_ERR_ALLOC;
  return hip_status(getrs<T>(h, n, nrhs, LU, lda, ipiv, B, ldb));
}

}  // namespace
}  // namespace lupp

extern "C" {

int lupp_create(lupp_handle_t* h) {
  if (!h) return -1;
  lupp_handle_st* p = new (std::nothrow) lupp_handle_st();
  if (!p) return LUPP_ERR_ALLOC;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = lupp::setup_batched(p);
  if (e != hipSuccess) {
    lupp::free_batched(p);
    delete p;
    return e == hipErrorOutOfMemory ? LUPP_ERR_ALLOC : lupp::hip_status(e);
  }
  *h = p;
  return LUPP_OK;
}

int lupp_destroy(lupp_handle_t h) {
  if (!h) return -1;
  int rc = LUPP_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) rc = lupp::hip_status(e);
  for (auto& r : h->records) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->bulk) (void)hipStreamSynchronize(h->bulk);
  if (h->side2) (void)hipStreamSynchronize(h->side2);
  if (h->bulk2) (void)hipStreamSynchronize(h->bulk2);
  if (h->look) (void)hipStreamSynchronize(h->look);
  if (h->look2) (void)hipStreamSynchronize(h->look2);
  for (hipEvent_t e : h->dag_events) (void)hipEventDestroy(e);
  if (h->ev_cols) (void)hipEventDestroy(h->ev_cols);
  if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
  if (h->ev_bulk) (void)hipEventDestroy(h->ev_bulk);
  if (h->ev_trsm) (void)hipEventDestroy(h->ev_trsm);
  for (int o = 0; o < 2; ++o)
    for (int e = 0; e < 4; ++e)
      if (h->tm_ev[o][e]) (void)hipEventDestroy(h->tm_ev[o][e]);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->bulk) (void)hipStreamDestroy(h->bulk);
  if (h->side2) (void)hipStreamDestroy(h->side2);
  if (h->bulk2) (void)hipStreamDestroy(h->bulk2);
  if (h->look) (void)hipStreamDestroy(h->look);
  if (h->look2) (void)hipStreamDestroy(h->look2);
  if (h->slots) (void)hipFree(h->slots);
  if (h->defer_buf) (void)hipFree(h->defer_buf);
  if (h->lp_scale[0]) (void)hipFree(h->lp_scale[0]);
  if (h->lp_pack[0]) (void)hipFree(h->lp_pack[0]);
  if (h->trsv.flags) (void)hipFree(h->trsv.flags);
  lupp::free_mixed(h);
  lupp::free_batched(h);
  lupp::free_qr(h);
  lupp::free_utv(h);
  delete h;
  return rc;
}

int lupp_set_stream(lupp_handle_t h, void* stream) {
  if (!h) return -1;
  h->stream = (hipStream_t)stream;
  return LUPP_OK;
}

int lupp_set_option(lupp_handle_t h, int option, int64_t value) {
  if (!h) return -1;
  switch (option) {
    case LUPP_OPT_NB:
      if (value < 1 || value > 1024) return -3;
      h->nb = value;
      return LUPP_OK;
    case LUPP_OPT_PANEL_LEAF:
      if (value < 16 || value > lupp::kBlockMaxWidth || value % 16 != 0) return -3;
      h->block = (int)value;
      return LUPP_OK;
    case LUPP_OPT_TIMING:
      if (value < 0 || value > 2) return -3;
      h->timing = (int)value;
      return LUPP_OK;
    case LUPP_OPT_LOOKAHEAD:
      if (value < 0 || value > 16) return -3;
      h->lookahead = (int)value;
      return LUPP_OK;
    case LUPP_OPT_UPDATE_PREC:
      if (value < LUPP_PREC_FP32 || value > LUPP_PREC_FP8_E4M3) return -3;
      h->update_prec = (int)value;
      return LUPP_OK;
    case LUPP_OPT_DEFER_SWAPS:
      if (value != 0 && value != 1) return -3;
      h->defer = (int)value;
      return LUPP_OK;
    case LUPP_OPT_SPLIT_UPDATE:
      if (value != 0 && value != 1) return -3;
      h->split = (int)value;
      return LUPP_OK;
    case LUPP_OPT_LP_PACKED:
      if (value != 0 && value != 1) return -3;
      h->lp_packed = (int)value;
      return LUPP_OK;
    default:
      return -2;
  }
}

int lupp_sync(lupp_handle_t h) {
  if (!h) return -1;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && h->side) e = hipStreamSynchronize(h->side);
  if (e == hipSuccess && h->bulk) e = hipStreamSynchronize(h->bulk);
  if (e == hipSuccess && h->side2) e = hipStreamSynchronize(h->side2);
  if (e == hipSuccess && h->bulk2) e = hipStreamSynchronize(h->bulk2);
  if (e == hipSuccess && h->look) e = hipStreamSynchronize(h->look);
  if (e == hipSuccess && h->look2) e = hipStreamSynchronize(h->look2);
  if (e != hipSuccess) return lupp::hip_status(e);
  if (h->slots) {
    int32_t err = 0;
    e = hipMemcpy(&err, &h->slots->err, sizeof(err), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lupp::hip_status(e);
    if (err) {
      const int32_t zero = 0;
      (void)hipMemcpy(&h->slots->err, &zero, sizeof(zero), hipMemcpyHostToDevice);
      (void)lupp::take_trsv_error(h);
      return LUPP_ERR_INTERNAL;
    }
  }
  if (h->qr && h->qr->slots) {
    int32_t qerr = 0;
    e = hipMemcpy(&qerr, &h->qr->slots->err, sizeof(qerr), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lupp::hip_status(e);
    if (qerr) {
      const int32_t zero = 0;
      (void)hipMemcpy(&h->qr->slots->err, &zero, sizeof(zero), hipMemcpyHostToDevice);
      return LUPP_ERR_INTERNAL;
    }
  }
  const int terr = lupp::take_trsv_error(h);
  if (terr < 0) return lupp::hip_status(hipGetLastError());
  int32_t sing = 0;
  if (h->trsv.sing) {
    e = hipMemcpy(&sing, h->trsv.sing, sizeof(sing), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lupp::hip_status(e);
    if (sing) {
      const int32_t zero = 0;
      (void)hipMemcpy(h->trsv.sing, &zero, sizeof(zero), hipMemcpyHostToDevice);
    }
  }
  if (terr) return LUPP_ERR_INTERNAL;
  if (sing) return LUPP_ERR_SINGULAR;
  return LUPP_OK;
}

int lupp_workspace_bytes(lupp_handle_t h, int op, int64_t m, int64_t n, int64_t k, size_t* bytes) {
  if (!h) return -1;
  if (op < LUPP_WS_DGETRF || op > LUPP_WS_BATCHED) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0 || (op == LUPP_WS_DGESV_MIXED && k > 60)) return -5;
  if (!bytes) return -6;
  const size_t base = sizeof(lupp::LeafSlots) + sizeof(lupp::SwapPairs);
  switch (op) {
    case LUPP_WS_DGETRF: *bytes = lupp::getrf_workspace_bytes(h, m, n, 8); break;
    case LUPP_WS_SGETRF: *bytes = lupp::getrf_workspace_bytes(h, m, n, 4); break;
    case LUPP_WS_DGETRS:
    case LUPP_WS_SGETRS: *bytes = base + lupp::trsv_workspace_bytes(n); break;
    case LUPP_WS_DGESV_MIXED: {
      const int saved = h->update_prec;
      h->update_prec = LUPP_PREC_FP16;  // the scale workspace of any low-precision format
      *bytes = lupp::getrf_workspace_bytes(h, n, n, 4) + lupp::trsv_workspace_bytes(n) +
               lupp::mixed_workspace_bytes(n, k < 1 ? 1 : k);
      h->update_prec = saved;
      break;
    }
    default: *bytes = lupp::batch_workspace_bytes(m); break;
  }
  return LUPP_OK;
}

int lupp_test_inject_fault(lupp_handle_t h, int what) {
  if (!h) return -1;
  if (what != 1 && what != 2) return -2;
  const hipError_t e = lupp::ensure_workspace(h);
  if (e != hipSuccess || lupp::ensure_trsv(h, 1) != hipSuccess) return LUPP_ERR_ALLOC;
  if (what == 1) {
    const hipError_t e1 = hipStreamSynchronize(h->stream);
    if (e1 != hipSuccess) return lupp::hip_status(e1);
    const int32_t one = 1;
    return lupp::hip_status(hipMemcpy(h->trsv.err, &one, sizeof(one), hipMemcpyHostToDevice));
  }
  h->trsv.tickets += (uint64_t)1 << 40;  // every ticket of the next solve falls below its base
  return LUPP_OK;
}

int lupp_timing_summary(lupp_handle_t h, int phase, int64_t* count, double* ms, double* flops, int reset) {
  if (!h) return -1;
  if (phase < LUPP_PHASE_PANEL || phase > LUPP_PHASE_PANEL_GEMM) return -2;
  if (!count) return -3;
  if (!ms) return -4;
  if (!flops) return -5;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && h->side) e = hipStreamSynchronize(h->side);
  if (e == hipSuccess && h->bulk) e = hipStreamSynchronize(h->bulk);
  if (e == hipSuccess && h->side2) e = hipStreamSynchronize(h->side2);
  if (e == hipSuccess && h->bulk2) e = hipStreamSynchronize(h->bulk2);
  if (e == hipSuccess && h->look) e = hipStreamSynchronize(h->look);
  if (e == hipSuccess && h->look2) e = hipStreamSynchronize(h->look2);
  if (e != hipSuccess) return lupp::hip_status(e);
  *count = 0;
  *ms = 0.0;
  *flops = 0.0;
  for (size_t i = 0; i < h->nrecords; ++i) {
    const lupp::TimingRecord& r = h->records[i];
    const bool match = (phase == LUPP_PHASE_UPDATE_BIG) ? (r.phase == LUPP_PHASE_UPDATE && r.big) : (r.phase == phase);
    if (!match) continue;
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess) return lupp::hip_status(e);
    *count += 1;
    *ms += t;
    *flops += r.flops;
  }
  if (reset) h->nrecords = 0;
  return LUPP_OK;
}

int lupp_timing_bytes(lupp_handle_t h, int phase, double* bytes) {
  if (!h) return -1;
  if (phase < LUPP_PHASE_PANEL || phase > LUPP_PHASE_PANEL_GEMM) return -2;
  if (!bytes) return -3;
  *bytes = 0.0;
  for (size_t i = 0; i < h->nrecords; ++i) {
    const lupp::TimingRecord& r = h->records[i];
    const bool match = (phase == LUPP_PHASE_UPDATE_BIG) ? (r.phase == LUPP_PHASE_UPDATE && r.big) : (r.phase == phase);
    if (match) *bytes += r.bytes;
  }
  return LUPP_OK;
}

const char* lupp_status_string(int status) {
  if (status == LUPP_OK) return "success";
  if (status < 0) return "invalid argument";
  if (status == LUPP_ERR_ALLOC) return "workspace allocation failed";
  if (status == LUPP_ERR_INTERNAL) return "device-side wait expired";
  if (status == LUPP_ERR_UNSUPPORTED) return "unsupported size or option";
  if (status == LUPP_ERR_SINGULAR) return "exactly singular triangular factor";
  if (status > LUPP_ERR_HIP && status < LUPP_ERR_ALLOC) return hipGetErrorString((hipError_t)(status - LUPP_ERR_HIP));
  return "unknown status";
}

int lupp_dgetrf(lupp_handle_t h, int64_t m, int64_t n, double* dA, int64_t lda, int32_t* dipiv, int32_t* dinfo) {
  return lupp::getrf_entry<double>(h, m, n, dA, lda, dipiv, dinfo);
}

int lupp_sgetrf(lupp_handle_t h, int64_t m, int64_t n, float* dA, int64_t lda, int32_t* dipiv, int32_t* dinfo) {
  return lupp::getrf_entry<float>(h, m, n, dA, lda, dipiv, dinfo);
}

int lupp_dgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const double* dLU, int64_t lda,
                const int32_t* dipiv, double* dB, int64_t ldb) {
  return lupp::getrs_entry<double>(h, trans, n, nrhs, dLU, lda, dipiv, dB, ldb);
}

int lupp_sgetrs(lupp_handle_t h, char trans, int64_t n, int64_t nrhs, const float* dLU, int64_t lda,
                const int32_t* dipiv, float* dB, int64_t ldb) {
  return lupp::getrs_entry<float>(h, trans, n, nrhs, dLU, lda, dipiv, dB, ldb);
}

}  // extern "C"
