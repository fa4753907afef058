// The handle and the host-side helpers shared by the driver sources.
#pragma once

#include <vector>

#include "common.h"

namespace lupp {
struct TimingRecord {
  hipEvent_t start = nullptr, stop = nullptr;
  int phase = 0;
  bool big = false;
  double flops = 0.0;
  double bytes = 0.0;  // algorithmic bytes (updates: C read and written, A and B read once)
};
struct MixedWs;
struct BatchWs;
struct UtvWs;
// Workspace of the QR path: the panel's exchange records, the explicit V,
// G, T, W and the partials of the row-chunked products.
struct QrWs {
  QrSlots* slots = nullptr;
  uint32_t epoch = 0;
  double* buf = nullptr;
  size_t bytes = 0;
  int64_t m = 0, n = 0;  // the shape the buffer layout is set for (last ensure_qr)
  // lookahead: the second V / G / -T^T and the per-stream scratch
  double* la = nullptr;
  size_t la_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // factored, T ready, next block, rest
};
}  // namespace lupp

struct lupp_handle_st {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t nb = 512;
  int block = 64;                   // widest column block factored in one cooperative launch
  lupp::LeafSlots* slots = nullptr;
  lupp::SwapPairs* pairs = nullptr;
  // deferred interchanges of the finished columns: per-step pairs, the gather
  // maps of all blocks, and 2*m ints of scratch (one allocation, grown on demand)
  void* defer_buf = nullptr;
  size_t defer_bytes = 0;
  int defer = 1;                    // defer the finished columns' interchanges when the workspace allows
  uint32_t epoch = 0;
  int timing = 0;  // LUPP_OPT_TIMING level
  std::vector<lupp::TimingRecord> records;  // events are created once and reused
  size_t nrecords = 0;
  int lookahead = 1;                // factor the next column block on a side stream
  hipStream_t side = nullptr;       // panel stream, restricted to panel_cus CUs
  hipStream_t bulk = nullptr;       // trailing-update stream, restricted to the other CUs
  int panel_cus = 0;                // CUs reserved for the panel while they overlap
  hipStream_t side2 = nullptr;      // the same pair for panels of up to 64 workgroups
  hipStream_t bulk2 = nullptr;
  hipStream_t look = nullptr;       // lookahead updates of the dataflow runtime, on the bulk CUs
  hipStream_t look2 = nullptr;      // the same beside the 64-CU panel stream
  int panel_cus2 = 0;
  int ncu = 0;                      // compute units of the device
  hipEvent_t ev_cols = nullptr;     // next block's columns updated (main -> side, bulk)
  hipEvent_t ev_panel = nullptr;    // next block factored (side -> main)
  hipEvent_t ev_bulk = nullptr;     // bulk update done (bulk -> main)
  hipEvent_t ev_trsm = nullptr;     // remaining columns interchanged and solved (bulk -> side)
  // split of the remaining-columns update between the bulk CUs and the panel's
  // CUs once the panel is done: sized from the panel time and the per-CU GEMM
  // rate, both measured on earlier steps (events read only once complete)
  int split = 1;
  hipEvent_t tm_ev[2][4] = {};      // per slot: panel start/end, bulk update start/end
  double tm_flops[2] = {0.0, 0.0};  // flops of that bulk update
  int tm_pair[2] = {0, 0};          // stream pair of that step (0: 32 panel CUs, 1: 64)
  bool tm_pending[2] = {false, false};
  int tm_slot = 0;
  double est_panel_ms[2] = {-1.0, -1.0};  // measured column-block time (ms) per pair, < 0 before the first
  double est_rate = -1.0;           // measured bulk GEMM flops per ms per CU, < 0 before the first
  int update_prec = 0;              // LUPP_PREC_* of sgetrf's trailing update
  // Workspace of the low-precision updates, one slot per update that may run
  // concurrently: 0 the next block's (caller's stream), 1 the bulk update,
  // 2 the bulk's share on the panel's CUs (loop) or the lookahead updates on
  // the first lookahead stream (dataflow runtime), 3 those on the second.
  int* lp_scale[4] = {nullptr, nullptr, nullptr, nullptr};  // block exponents
  int64_t lp_scale_cap = 0;         // ints in each lp_scale slot
  void* lp_pack[4] = {nullptr, nullptr, nullptr, nullptr};  // packed operands
  size_t lp_pack_cap = 0;           // bytes in each lp_pack slot
  int lp_packed = 1;                // LUPP_OPT_LP_PACKED
  std::vector<hipEvent_t> dag_events;  // task completion events of the dataflow runtime (reused)
  lupp::TrsvState trsv{};           // one-launch triangular solve state (flags on demand)
  lupp::MixedWs* mixed = nullptr;   // workspace of lupp_dgesv_mixed
  lupp::BatchWs* batch = nullptr;   // workspace and streams of the batched path
  lupp::QrWs* qr = nullptr;         // workspace of the Householder QR
  lupp::UtvWs* utv = nullptr;       // workspace of randUTV
};

namespace lupp {

inline int hip_status(hipError_t e) { return e == hipSuccess ? LUPP_OK : LUPP_ERR_HIP + (int)e; }

#define LUPP_TRY(expr)               \
  do {                               \
    hipError_t e_ = (expr);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Handle workspace of the factorization (slots, swap pairs, lookahead streams).
hipError_t ensure_workspace(lupp_handle_t h);
// Scale workspace of the low-precision update for an m x n factorization.
// Workspace of the deferred interchanges for an m x n factorization with the
// handle's nb; false when the deferral does not apply (the interchanges are
// then applied to the finished columns at every step).
bool ensure_defer(lupp_handle_t h, int64_t m, int64_t n, size_t elem);
// Streams of the dataflow runtime's lookahead updates (on first use).
bool ensure_look_streams(lupp_handle_t h);
hipError_t ensure_lp_scale(lupp_handle_t h, int64_t m, int64_t n, int64_t nb);
// Flags of the one-launch triangular solve for n rows.
hipError_t ensure_trsv(lupp_handle_t h, int64_t n);
// The factorization and the solve on the handle's stream (arguments checked).
template <typename T>
hipError_t getrf(lupp_handle_t h, int64_t m, int64_t n, T* A, int64_t lda, int32_t* ipiv, int32_t* info);
template <typename T>
hipError_t getrs(lupp_handle_t h, int64_t n, int64_t nrhs, const T* LU, int64_t lda, const int32_t* ipiv, T* B,
                 int64_t ldb);
void free_mixed(lupp_handle_t h);
void free_batched(lupp_handle_t h);
void free_qr(lupp_handle_t h);
void free_utv(lupp_handle_t h);
// Householder QR of an m x n matrix on the handle's stream (arguments checked).
hipError_t geqrf(lupp_handle_t h, int64_t m, int64_t n, double* A, int64_t lda, double* tau);
size_t qr_workspace_bytes(int64_t m, int64_t n);
// QR workspace laid out for an m x n problem (grown on demand).
hipError_t ensure_qr(lupp_handle_t h, int64_t m, int64_t n);
// One 128-column outer block of the Householder QR (see qr.hip); V (r x 128,
// ld r) at qr_v(h) and -T^T (128 x 128) at qr_tneg(h) afterwards.
hipError_t qr_outer(lupp_handle_t h, int64_t r, int64_t ncols, double* A, int64_t lda, double* tau, int64_t B,
                    bool keep_wy);
// out (ldw x N) = V^T X, V r x ldw (ldw 32, 64 or 128); part: chunk partials.
hipError_t qr_tn(hipStream_t s, int64_t r, int64_t N, const double* V, int64_t ldv, const double* X, int64_t ldx,
                 int ldw, double* part, double* out, int64_t chunk_width = 0);
inline double* qr_v(lupp_handle_t h);
inline double* qr_tneg(lupp_handle_t h);
inline double* qr_part(lupp_handle_t h);
int timer_begin(lupp_handle_t h, int phase, hipStream_t st);
void timer_end(lupp_handle_t h, int idx, hipStream_t st, double flops, bool big = false, double bytes = 0.0);
// Batched path set-up at handle creation: class streams and events, grids, and
// the device address of the allocation-free entry point's scratch array.
hipError_t setup_batched(lupp_handle_t h);

}  // namespace lupp

namespace lupp {
// After the stream has drained: read and clear the triangular solve's error
// flag; when it was set, the host's ticket count is re-read from the device
// counter, so that later solves start in step.  Returns the flag (0 none,
// 1 an expired wait, 2 a ticket mismatch) or -1 if the copies failed.
int take_trsv_error(lupp_handle_t h);
// Device bytes the handle holds for these calls with its current options.
size_t getrf_workspace_bytes(lupp_handle_t h, int64_t m, int64_t n, size_t elem);
size_t trsv_workspace_bytes(int64_t n);
size_t mixed_workspace_bytes(int64_t n, int64_t restart);
size_t batch_workspace_bytes(int64_t batch);
}  // namespace lupp

namespace lupp {
// Views into the QR workspace (layout of qr_outer: V, G, -T^T, G32, T32, W,
// W2, chunk partials).
inline double* qr_v(lupp_handle_t h) { return h->qr->buf; }
inline double* qr_tneg(lupp_handle_t h) { return h->qr->buf + 128 * h->qr->m + 128 * 128; }
inline double* qr_part(lupp_handle_t h) {
  const int64_t nn = h->qr->n > 128 ? h->qr->n : 128;
  return h->qr->buf + 128 * h->qr->m + 2 * 128 * 128 + 2 * 32 * 32 + 2 * 128 * nn;
}
}  // namespace lupp
