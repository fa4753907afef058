// Wavefront-level helpers shared by the device sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace lupp
