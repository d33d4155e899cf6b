// Fused single-launch FP32 solve (stage setup + Riccati factor + all ADMM
// iterations in one workgroup per agent, operators resident on chip).
#pragma once

#include <hip/hip_runtime.h>

#include "mpc_internal.h"

namespace mpc {

// True if the fused kernel has an instantiation for this uniform shape.
bool fused_supported(int N, int nx, int nu, int n_feet);
// Threads per workgroup and dynamic LDS bytes of the fused kernel for the shape.
void fused_launch_shape(int N, int nx, int nu, int n_feet, int* threads, size_t* lds);
hipError_t fused_solve_f32(const AgentDesc* d_desc, int n_agents, int N, int nx, int nu,
                           int n_feet, Inputs<float> in, SolverConsts sc, int iters, int warm,
                           State<float> st, int threads, size_t lds, hipStream_t stream);

}  // namespace mpc
