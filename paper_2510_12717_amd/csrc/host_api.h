// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mpc.h"

namespace mpc {

// Records msg as this thread's last error (mpc_last_error) and returns s.
mpc_status api_fail(mpc_status s, const std::string& msg);

// Precisions whose factor products run in a lower or matrix-core precision
// with refinement sweeps in the iterations, and their product selector of the
// factor kernel (1 BF16, 2 FP16, 3 FP32 operands).
inline bool refine_precision(int precision) {
  return precision == MPC_BF16_REFINE || precision == MPC_FP16_REFINE || precision == MPC_FP32_REFINE;
}
inline int refine_product(int precision) {
  return precision == MPC_BF16_REFINE ? 1 : precision == MPC_FP16_REFINE ? 2 : 3;
}

}  // namespace mpc

#define MPC_HIP_TRY(expr)                                                                   \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return ::mpc::api_fail(                                                               \
          _e == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,                  \
          std::string(#expr) + ": " + hipGetErrorString(_e));                              \
  } while (0)
