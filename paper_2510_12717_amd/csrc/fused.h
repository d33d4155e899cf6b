// Register-resident FP32 solve: an FP64 MFMA Riccati-factor kernel followed
// by an iteration kernel that keeps every stage's operators in the VGPRs of
// one wavefront per stage (horizons up to 11), or of one wavefront per two
// stages with the closed-loop operators streamed through LDS (12 to 20).
#pragma once

#include <hip/hip_runtime.h>

#include "mpc_internal.h"

namespace mpc {

// True if the register-resident kernels have an instantiation for this shape
// (with nc no-slip rows per state: the register-resident body, 2 <= N <= 11,
// within the LDS).
bool fused_supported(int N, int nx, int nu, int n_feet, int nc = 0);
// Horizon bucket of the register-resident launch groups: horizons up to 6 share
// a launch of at most 7 wavefronts per agent (two agents fit one compute
// unit), 7 to 11 a launch of up to 12, and 12 to 20 the streaming kernel's.
inline int fused_bucket(int N) { return N <= 6 ? 0 : N <= 11 ? 1 : 2; }
// Threads per workgroup and dynamic LDS bytes of the iteration kernel for a
// launch whose longest horizon is N.
void fused_launch_shape(int N, int nx, int nu, int n_feet, int* threads, size_t* lds, int nc = 0);
// Floats of operator workspace one agent of this shape class needs.
size_t fused_agent_floats(int N, int nx, int nu);
// Raise the dynamic-LDS limits of every register-resident kernel (once per device).
hipError_t fused_set_limits();
// Launch for the n_launch agents list[0..n_launch) (all of one shape class,
// horizons at most N).  phase_mask: 1 = factor kernel, 2 = iteration kernel.
// counter (device int, or nullptr): the iterations run as one persistent
// launch over the whole list, every horizon, agents taken from the counter.
// f32_products: the factor's block products on the FP32 matrix cores.
// nc: no-slip rows per state (in.J and st.zc / st.yc set; not persistent).
hipError_t fused_solve_f32(const AgentDesc* d_desc, const int32_t* list, int n_launch, int N, int nx,
                           int nu, int n_feet, Inputs<float> in, SolverConsts sc, int iters,
                           int warm, State<float> st, float* fws, hipStream_t stream,
                           int phase_mask, int* counter = nullptr, bool f32_products = false,
                           int nc = 0);
// Workgroup size and dynamic LDS of the persistent launch for longest horizon N.
void fused_persistent_shape(int N, int nx, int nu, int n_feet, int* threads, size_t* lds);

// The same factor kernel writing the generic operator layout at ws + ows (any
// horizon): block products in FP64 (prod 0), or BF16 (1) / FP16 (2) operands
// on the matrix cores with FP32 accumulation for the mixed-precision plans;
// the stage-Hessian inverse is FP64 in every case.
bool mixed_supported(int nx, int nu);
hipError_t launch_mixed_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, int nx,
                               int nu, int prod, Inputs<float> in, SolverConsts sc, float* ws,
                               int32_t* status, hipStream_t stream);

}  // namespace mpc
