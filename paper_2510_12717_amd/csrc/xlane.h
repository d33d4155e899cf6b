// Cross-lane moves of one wavefront without the LDS crossbar (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace mpc {

// DPP within rows of 16 lanes: the value of the lane that control word C
// names (quad_perm, row_ror, row_half_mirror, ...); every lane is active.
template <int C>
__device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, 0xF, 0xF, false));
}
template <int C>
__device__ inline double dpp(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), C, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// All-reduce over aligned groups of 4 lanes (quad_perm [1,0,3,2], [2,3,0,1]).
template <typename T>
__device__ inline T quad_sum(T v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  return v;
}

}  // namespace mpc
