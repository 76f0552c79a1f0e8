// Wavefront-level helpers shared by the one-workgroup factorisation kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace ttr {

// DPP move of a double within a row of 16 lanes (CTRL: the DPP control word;
// every lane's source lies in its own row, so no lane reads out of range and
// the move needs no prior value in its destination)
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const long long x = __double_as_longlong(v);
  int lo = (int)(x & 0xffffffffll), hi = (int)(x >> 32);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP row broadcast of a double to the rows of ROWMASK: row_bcast:15 (0x142)
// sends lane 15 of each row to the next row, row_bcast:31 (0x143) sends lane
// 31 to rows 2 and 3; lanes of rows outside ROWMASK read 0
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_row_bcast(double v) {
  const long long x = __double_as_longlong(v);
  int lo = (int)(x & 0xffffffffll), hi = (int)(x >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of lane T of each quad of lanes, in all four (quad_perm [T,T,T,T])
template <int T>
__device__ __forceinline__ double quad_bcast(double v) {
  return dppd<T * 0x55>(v);
}

// sum over each quad of lanes, in all four (quad_perm [1,0,3,2], [2,3,0,1])
__device__ __forceinline__ double quad_sum(double v) {
  v += dppd<0xB1>(v);
  return v + dppd<0x4E>(v);
}

// value of lane `lane` (wavefront-uniform) in every lane
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

}  // namespace ttr
