/*
 * Philox-4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), arranged to emit the
 * same stream as numpy's Philox bit generator with key = (k0, k1) and a zero
 * starting counter: block b (b = 0, 1, ...) is the 10-round bijection of the
 * counter value b + 1, and its four 64-bit words are draws 4b .. 4b+3.
 * U(0,1) doubles are (word >> 11) * 2^-53.
 *
 * Input generation only: this file holds none of the factorization's
 * arithmetic.  Element e of the output is draw e0 + e, so any range of the
 * stream can be produced independently (the fills below split it over
 * threads).
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

static inline void mulhilo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

static inline void philox_block(uint64_t ctr0, uint64_t ctr1, uint64_t k0, uint64_t k1, uint64_t out[4]) {
  uint64_t c0 = ctr0, c1 = ctr1, c2 = 0, c3 = 0;
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo(PHILOX_M0, c0, &hi0, &lo0);
    mulhilo(PHILOX_M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* draw d of the stream (0-based) */
static inline uint64_t draw(uint64_t k0, uint64_t k1, uint64_t d, uint64_t* cache_blk, uint64_t cache[4]) {
  uint64_t blk = d >> 2;
  if (blk != *cache_blk) {
    uint64_t ctr = blk + 1; /* counter is incremented before each block */
    philox_block(ctr, ctr == 0 ? 1 : 0, k0, k1, cache);
    *cache_blk = blk;
  }
  return cache[d & 3];
}

/* out[e] = U(0,1) draw (e0 + e), e in [0, count) */
void synth_u01(uint64_t k0, uint64_t k1, uint64_t e0, double* out, int64_t count, int nthreads) {
  (void)nthreads;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    uint64_t cache_blk = UINT64_MAX, cache[4];
#pragma omp for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
      uint64_t w = draw(k0, k1, e0 + (uint64_t)e, &cache_blk, cache);
      out[e] = (double)(w >> 11) * (1.0 / 9007199254740992.0);
    }
  }
}

/* out[e] = a * U(0,1) + b for the exact maps used by the recipes (a = 2, b = -1
 * or a = 1, b = -0.5): both are exact in binary64 */
void synth_affine_u01(uint64_t k0, uint64_t k1, uint64_t e0, double* out, int64_t count, double a, double b,
                      int nthreads) {
  (void)nthreads;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    uint64_t cache_blk = UINT64_MAX, cache[4];
#pragma omp for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
      uint64_t w = draw(k0, k1, e0 + (uint64_t)e, &cache_blk, cache);
      double u = (double)(w >> 11) * (1.0 / 9007199254740992.0);
      out[e] = u * a + b;
    }
  }
}
