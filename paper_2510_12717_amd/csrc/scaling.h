// Ruiz equilibration (Alg. 1's scaling step) and the adaptive-rho update on
// the device; kernels in scaling.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "mpc_internal.h"

namespace mpc {

// Per-agent scale record (doubles): D_x [0, 64), D_u [64, 96), cost factor at 96.
constexpr int kScaleStride = 128, kScaleDu = 64, kScaleC = 96;

// Where the scaled problem data go (same layouts and offsets as the caller's).
template <typename T>
struct ScaledInputs {
  T *A, *B, *c, *q, *r, *xr, *x0, *tau, *mu;
};

// Equilibrate every agent (rounds of Ruiz), write the scaled data and the scale
// record, and move a warm start (u, z, y in st) into the scaled variables.
template <typename T>
hipError_t launch_ruiz(const AgentDesc* d_desc, int n, Inputs<T> in, int rounds, ScaledInputs<T> out,
                       double* scale, int warm, State<T> st, hipStream_t stream);
// Map the iterate (x, u, z, y in st) back to the original variables.
template <typename T>
hipError_t launch_unscale(const AgentDesc* d_desc, int n, const double* scale, State<T> st,
                          hipStream_t stream);
// Replace rho[a] by its residual-balancing estimate where it moved by more than
// tol either way; res holds the residual kernel's output for the problem in `in`.
// The rho the next segment runs with goes to hist[a * n_seg + seg].
template <typename T>
hipError_t launch_rho_update(const AgentDesc* d_desc, int n, Inputs<T> in, State<T> st,
                             const double* res, double* rho, double tol, double* hist, int n_seg,
                             int seg, hipStream_t stream);
// rho[a] = x and hist[a * n_seg] = x for every agent.
hipError_t launch_rho_init(double* rho, double* hist, int n, int n_seg, double x, hipStream_t stream);

}  // namespace mpc
