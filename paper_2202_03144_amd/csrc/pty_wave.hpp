// Wavefront-wide reductions for gfx950 (wave64) through DPP lane moves.
#pragma once
#include <hip/hip_runtime.h>

namespace pty {

// Wavefront reductions through DPP lane moves (VALU only, no LDS round
// trips): quad swaps, half-row and row mirrors, then row broadcasts 15 and
// 31, after which lane 63 holds the result over all 64 lanes; fixed order.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_or_zero(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}
// maximum of non-negative floats (their bit patterns order like integers)
__device__ __forceinline__ float wave_max_nonneg(float x) {
  unsigned v = __float_as_uint(x);
  v = max(v, (unsigned)dpp_or_zero<0xB1, 0xf>((int)v));    // quad_perm [1, 0, 3, 2]
  v = max(v, (unsigned)dpp_or_zero<0x4E, 0xf>((int)v));    // quad_perm [2, 3, 0, 1]
  v = max(v, (unsigned)dpp_or_zero<0x141, 0xf>((int)v));   // row_half_mirror
  v = max(v, (unsigned)dpp_or_zero<0x140, 0xf>((int)v));   // row_mirror
  v = max(v, (unsigned)dpp_or_zero<0x142, 0xa>((int)v));   // row_bcast:15
  v = max(v, (unsigned)dpp_or_zero<0x143, 0xc>((int)v));   // row_bcast:31
  return __uint_as_float((unsigned)__builtin_amdgcn_readlane((int)v, 63));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_or_zero_d(double x) {
  const int lo = dpp_or_zero<CTRL, ROWMASK>(__double2loint(x));
  const int hi = dpp_or_zero<CTRL, ROWMASK>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_or_zero_d<0xB1, 0xf>(v);
  v += dpp_or_zero_d<0x4E, 0xf>(v);
  v += dpp_or_zero_d<0x141, 0xf>(v);
  v += dpp_or_zero_d<0x140, 0xf>(v);
  v += dpp_or_zero_d<0x142, 0xa>(v);
  v += dpp_or_zero_d<0x143, 0xc>(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

}  // namespace pty
