// Wave-level reductions shared by the latency-bound kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace rif {

// Sum over the 64 lanes (all active), the same bits in every lane and every
// call: within each row of 16 lanes by DPP moves (swap neighbours, swap
// pairs, rotate by 4, rotate by 8), then the four row sums read from lanes 0,
// 16, 32, 48 and added in that order.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x += dpp_move<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp_move<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp_move<0x124>(x);   // row_ror:4
  x += dpp_move<0x128>(x);   // row_ror:8
  return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

// Max over the 64 lanes (all active) of doubles (NaN lanes ignored, as fmax
// does) and min of ints, every lane getting the result; both are
// order-free, so every wave gets the same value.
__device__ __forceinline__ double wave_max_dpp(double x) {
  x = fmax(x, dpp_move<0xB1>(x));
  x = fmax(x, dpp_move<0x4E>(x));
  x = fmax(x, dpp_move<0x124>(x));
  x = fmax(x, dpp_move<0x128>(x));
  return fmax(fmax(lane_value(x, 0), lane_value(x, 16)), fmax(lane_value(x, 32), lane_value(x, 48)));
}
__device__ __forceinline__ int wave_min_int_dpp(int x) {
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
  return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

}  // namespace rif
