// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mpc.h"

namespace mpc {

// Records msg as this thread's last error (mpc_last_error) and returns s.
mpc_status api_fail(mpc_status s, const std::string& msg);

}  // namespace mpc

#define MPC_HIP_TRY(expr)                                                                   \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return ::mpc::api_fail(                                                               \
          _e == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,                  \
          std::string(#expr) + ": " + hipGetErrorString(_e));                              \
  } while (0)
