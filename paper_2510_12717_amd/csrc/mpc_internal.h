// Internal declarations shared by the HIP translation units of the solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

// Per-agent shape and offsets.  Input offsets index the caller's arrays
// (elements from each Inputs base pointer), solution offsets index the
// resident x/u/z/y, and ws is the element offset of the agent's factor
// workspace.  flags bit 0: warm start this agent when a launch passes warm < 0.
struct AgentDesc {
  int32_t N, nx, nu, n_tau, n_feet, foot_dim, m, flags;
  int64_t oA, oB, oc, oq, orr, oxr, ox0, otau, ost, omu, our;
  int64_t ox, ou, oz, oy;
  int64_t ows;  // generic-kernel factor workspace (elements of the io type)
  int64_t ofw;  // register-resident workspace (floats), -1 if the agent has none
  // no-slip rows (plans with them): Jacobian rows [n_feet*foot_dim][nx] and
  // the rows' (z_c, y_c) [N][n_feet*foot_dim]
  int64_t oJ = 0, ozc = 0;
};

struct SolverConsts {
  double rho, sigma, alpha, rho_eq, rho_min;
  const double* rho_agent = nullptr;  // per-agent rho (adaptive rho), or null: rho for all
};

// The constants one agent runs with (its own rho when the plan adapts rho).
__host__ __device__ inline SolverConsts agent_consts(const SolverConsts& sc, int agent) {
  SolverConsts s = sc;
  if (sc.rho_agent) s.rho = sc.rho_agent[agent];
  return s;
}

template <typename T>
struct Inputs {
  const T *A, *B, *c, *q, *r, *xr, *x0, *tau, *mu;
  const uint8_t* st;
  const T* uref;  // may be null
  // joint limits x_lo <= x_k <= x_hi (k = 1..N), [nx] per agent at the q offset;
  // null: no state rows
  const T* xlo = nullptr;
  const T* xhi = nullptr;
  // no-slip rows J_f v_k = 0 of feet in stance (k = 1..N): the rows
  // [n_feet*foot_dim][nx] per agent at the oJ offset; null: none
  const T* J = nullptr;
};

template <typename T>
struct State {
  T *x, *u, *z, *y;
  T* obj;
  double* res;
  int32_t* status;
  // the joint-limit rows' (z_x, y_x), [N][nx] per agent at the c offset (with limits)
  T* zx = nullptr;
  T* yx = nullptr;
  // the no-slip rows' (z_c, y_c), [N][n_feet*foot_dim] per agent at the ozc offset
  T* zc = nullptr;
  T* yc = nullptr;
};

enum : int32_t { AGENT_OK = 0, AGENT_CONVERGED = 1, AGENT_NOT_PD = 2, AGENT_NONFINITE = 3 };
enum : int32_t { AGENT_FLAG_WARM = 1 };

// Warm start of one agent: the launch's flag, or the agent's own when warm < 0.
__host__ __device__ inline bool agent_warm(int warm, const AgentDesc& d) {
  return warm < 0 ? (d.flags & AGENT_FLAG_WARM) != 0 : warm != 0;
}

// Elements of factor workspace per agent for the generic kernels:
// K [N][nu][nx], Acl [N][nx][nx], Hinv [N][nu][nu], s [N][nx], l/h/rho [N][m].
inline int64_t generic_ws_elems(int N, int nx, int nu, int m) {
  return (int64_t)N * ((int64_t)nu * nx + (int64_t)nx * nx + (int64_t)nu * nu + nx + 3 * m);
}

inline size_t generic_factor_lds(int nx, int nu, size_t esz) {
  (void)esz;  // the recursion runs in double whatever the io type
  return 8 * (size_t)(nu * nu + 3 * nx * nx + 3 * nx * nu + nu + 64);
}
inline size_t generic_admm_lds(int N, int nx, int nu, int m, size_t esz, bool limits = false,
                               int nc = 0) {
  (void)esz;  // vectors are held in double whatever the io type
  // + 256 doubles of reduction scratch for the refinement's stopping test
  // (+ the joint-limit rows' z_x, y_x; + the no-slip rows' z_c, y_c and
  // y_c - rho_c z_c)
  return 8 * (size_t)(2 * (N + 1) * nx + 4 * N * nu + 2 * N * m + 3 * N * nx + nx + N * nu + 256 +
                      (limits ? 2 * N * nx : 0) + 3 * N * nc);
}
// Residual kernel: costates and x ((N+1) x nx each) and u (N x nu) in double,
// then stage k's A_k and B_k staged in the io type with rows padded by one
// element.
inline size_t generic_residual_lds(int N, int nx, int nu, size_t esz) {
  const size_t dbl = 8 * (2 * (size_t)(N + 1) * nx + (size_t)N * nu);
  return dbl + esz * ((size_t)nx * (nx + 1) + (size_t)nx * (nu + 1)) + 16;
}

// The paper-form inner solve (quasi-definite KKT factored by LDL^T, finite
// rho_eq): S_k^{-1} of every stage, [N][nu+nx][nu+nx] per agent (io type).
inline int64_t kkt_ws_elems(int N, int nx, int nu) {
  return (int64_t)N * (nu + nx) * (nu + nx);
}
inline size_t kkt_factor_lds(int nx, int nu, int m) {
  const size_t nw = (size_t)(nu + nx);
  return 8 * (nw * nw + 4 * (size_t)nx * nx + 2 * (size_t)nu * nx + (size_t)m);
}
inline size_t kkt_admm_lds(int N, int nx, int nu, int m) {
  return 8 * ((size_t)(N + 1) * nx + (size_t)N * nu + 2 * (size_t)N * m + 2 * (size_t)N * nx +
              2 * (size_t)N * (nu + nx) + 3 * (size_t)nx);
}
hipError_t kkt_set_lds_limits(size_t lds_factor, size_t lds_admm);

// The generic Riccati factor as a parallel-in-time scan (kernels_scan.hip):
// element buffers E0, E1 of scan_elements_bytes each for the launch list.
size_t scan_elements_bytes(int n_agents, int Nmax, int nx);
template <typename T>
hipError_t launch_scan_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, int Nmax, int nx,
                              int nu, int m, Inputs<T> in, SolverConsts sc, T* ws, double* E0, double* E1,
                              int32_t* status, size_t lds_ops, hipStream_t s);
hipError_t scan_set_limits();
template <typename T>
hipError_t launch_kkt_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                             SolverConsts sc, T* ws, int32_t* status, size_t lds,
                             hipStream_t stream);
// zd, yd: the dynamics rows' (z, y), [N][nx] per agent at the c offset.
template <typename T>
hipError_t launch_kkt_admm(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                           SolverConsts sc, int iters, int warm, const T* ws, State<T> st,
                           T* zd, T* yd, size_t lds, hipStream_t stream);

// Raise the dynamic-LDS limit of the generic kernels to what a plan needs.
hipError_t generic_set_lds_limits(size_t lds_factor, size_t lds_admm, size_t lds_res);

// Launchers (generic kernels, one workgroup per agent).  list (nullable) maps
// workgroup i to agent list[i]; n_launch workgroups are launched.
template <typename T>
hipError_t launch_generic_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch,
                                 Inputs<T> in, SolverConsts sc, T* ws, int32_t* status, size_t lds,
                                 int threads, hipStream_t stream);
// sweeps >= 0 selects the mixed-precision iteration: rollout under the exact
// dynamics and up to `sweeps` KKT-residual refinement sweeps per x-update,
// stopping once |r|_inf <= rtol * |b|_inf.  sweeps < 0: plain iteration.
template <typename T>
hipError_t launch_generic_admm(const AgentDesc* d_desc, const int32_t* list, int n_launch,
                               Inputs<T> in, SolverConsts sc, int iters, int warm, const T* ws,
                               State<T> st, size_t lds, int threads, hipStream_t stream,
                               int sweeps = -1, double rtol = 0.0);
template <typename T>
hipError_t launch_residual(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                           SolverConsts sc, State<T> st, size_t lds, hipStream_t stream);
template <typename T>
hipError_t launch_advance(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                          const T* u, const T* noise, T* x0_next, hipStream_t stream);

}  // namespace mpc
