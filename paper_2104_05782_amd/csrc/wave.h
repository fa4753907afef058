// Wavefront-level helpers shared by the device sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lupp {

// Wavefront argmax of (|a|, row) under the total order (|a| desc, row asc).
// |a| >= 0, so its binary64 pattern read as an unsigned integer is ordered
// like the value.  Four DPP steps (partners lane^1, lane^2, the mirror inside
// 8 lanes, the mirror inside 16) leave every lane with its 16-lane row's
// winner; the four row winners are then read as uniform values and combined.
// No LDS round trip (ds_bpermute) is involved.
__device__ __forceinline__ bool key_better(uint32_t hi, uint32_t lo, uint32_t idx, uint32_t bhi, uint32_t blo,
                                           uint32_t bidx) {
  return hi > bhi || (hi == bhi && (lo > blo || (lo == blo && idx < bidx)));
}

template <int CTRL>
__device__ __forceinline__ void dpp_step(uint32_t& hi, uint32_t& lo, uint32_t& idx) {
  const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, 0xF, 0xF, false);
  const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, 0xF, 0xF, false);
  const uint32_t oidx = (uint32_t)__builtin_amdgcn_update_dpp((int)idx, (int)idx, CTRL, 0xF, 0xF, false);
  if (key_better(ohi, olo, oidx, hi, lo, idx)) {
    hi = ohi;
    lo = olo;
    idx = oidx;
  }
}

// returns the wavefront's winner in every lane (value as double, row index)
__device__ __forceinline__ void wave_argmax(double& v, int64_t& i) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  uint32_t hi = (uint32_t)(bits >> 32), lo = (uint32_t)bits;
  // an empty candidate (v < 0) must lose to any real one: map it to key 0 and
  // the largest index
  uint32_t idx = (v < 0.0 || i >= INT32_MAX) ? 0xFFFFFFFFu : (uint32_t)i;
  if (v < 0.0) hi = lo = 0;
  dpp_step<0xB1>(hi, lo, idx);   // quad_perm(1,0,3,2)
  dpp_step<0x4E>(hi, lo, idx);   // quad_perm(2,3,0,1)
  dpp_step<0x141>(hi, lo, idx);  // row_half_mirror
  dpp_step<0x140>(hi, lo, idx);  // row_mirror
  uint32_t bhi = __builtin_amdgcn_readlane(hi, 0), blo = __builtin_amdgcn_readlane(lo, 0),
           bidx = __builtin_amdgcn_readlane(idx, 0);
#pragma unroll
  for (int rrow = 1; rrow < 4; ++rrow) {
    const uint32_t h2 = __builtin_amdgcn_readlane(hi, rrow * 16), l2 = __builtin_amdgcn_readlane(lo, rrow * 16),
                   i2 = __builtin_amdgcn_readlane(idx, rrow * 16);
    if (key_better(h2, l2, i2, bhi, blo, bidx)) {
      bhi = h2;
      blo = l2;
      bidx = i2;
    }
  }
  if (bidx == 0xFFFFFFFFu) {
    v = -1.0;
    i = INT64_MAX;
  } else {
    v = __longlong_as_double((long long)(((uint64_t)bhi << 32) | blo));
    i = (int64_t)bidx;
  }
}

// readlane of a 64-bit or 32-bit value (k wave-uniform)
__device__ __forceinline__ double readlane_d(double v, int k) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float readlane_d(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// DPP partner values inside 16-lane rows (quad_perm / row_half_mirror /
// row_mirror), for 64-bit and 32-bit lanes
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)u, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(u >> 32), (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

// wavefront max of doubles (NaN ignored), the same value in every lane
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  double m = readlane_d(v, 0);
  m = fmax(m, readlane_d(v, 16));
  m = fmax(m, readlane_d(v, 32));
  return fmax(m, readlane_d(v, 48));
}

// wavefront min of unsigned ints, the same value in every lane
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<0xB1>(v));
  v = min(v, dpp_u32<0x4E>(v));
  v = min(v, dpp_u32<0x141>(v));
  v = min(v, dpp_u32<0x140>(v));
  uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
  m = min(m, (uint32_t)__builtin_amdgcn_readlane((int)v, 16));
  m = min(m, (uint32_t)__builtin_amdgcn_readlane((int)v, 32));
  return min(m, (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
}

// Lane k's value in every lane of its 16-lane row (DPP row broadcast).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x150 + K, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x150 + K, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <int K>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + K, 0xF, 0xF, false));
}

// Workgroup barrier that waits only for LDS traffic.  (__syncthreads also
// waits for every outstanding global load and store of the wave, which would
// put a memory round trip on each step.)  The signal fences keep the compiler
// from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt untouched
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int K, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (K < N) {
    f(std::integral_constant<int, K>());
    static_for<K + 1, N>(f);
  }
}

// f(integral_constant<c>) for a wave-uniform runtime c in [LO, HI): a
// balanced tree of scalar branches, so that register arrays are indexed with
// compile-time subscripts only.
template <int LO, int HI, typename F>
__device__ __forceinline__ void dispatch(int c, F&& f) {
  if constexpr (HI - LO == 1) {
    f(std::integral_constant<int, LO>());
    // an empty asm statement with the leaf's constant keeps the optimizer
    // from merging the leaves into one access at a computed offset (which
    // would move the register array to scratch memory)
    __asm__ volatile("; leaf %0" ::"n"(LO));
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (c < MID)
      dispatch<LO, MID>(c, f);
    else
      dispatch<MID, HI>(c, f);
  }
}

}  // namespace lupp
