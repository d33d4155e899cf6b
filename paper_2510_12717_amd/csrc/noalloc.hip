// mpc_solve_noalloc: the solve of a uniform FP32 batch without a plan and
// without any device allocation, for callers that cannot allocate (work
// recorded under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The per-agent descriptors, the launch list and the
// register-resident operator workspace live in one file-scope device array;
// the caller's solution buffers hold the iterate.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/mpc.h"
#include "fused.h"
#include "host_api.h"
#include "mpc_internal.h"

using namespace mpc;

namespace {

constexpr int kMaxDevices = 64;

// Scratch of the no-allocation entry point: one copy per device, held until
// the process ends.  Host code never passes the array's name to a kernel or
// a copy; it uses the device address resolved once per device below.
__device__ __align__(256) unsigned char scratch[MPC_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (resolved on the first call made
// with the device current).
mpc_status scratch_ptr(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return api_fail(MPC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    // the kernel limits are per process and per device: raise them once here
    hipError_t le = fused_set_limits();
    if (le != hipSuccess)
      return api_fail(MPC_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(le));
    g_ptr[device] = ptr;
  }
  *out = g_ptr[device];
  return MPC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Descriptors of n agents of one shape stored back to back, and the identity
// launch list.
__global__ void k_uniform_desc(mpc_shape s, int n, int64_t fws_per_agent, AgentDesc* out,
                               int32_t* list) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int m = s.nu + 4 * s.n_feet;
  AgentDesc d;
  d.N = s.N;
  d.nx = s.nx;
  d.nu = s.nu;
  d.n_tau = s.n_tau;
  d.n_feet = s.n_feet;
  d.foot_dim = s.foot_dim;
  d.m = m;
  d.flags = 0;
  d.oA = (int64_t)a * s.N * s.nx * s.nx;
  d.oB = (int64_t)a * s.N * s.nx * s.nu;
  d.oc = (int64_t)a * s.N * s.nx;
  d.oq = (int64_t)a * s.nx;
  d.orr = (int64_t)a * s.nu;
  d.oxr = (int64_t)a * (s.N + 1) * s.nx;
  d.ox0 = (int64_t)a * s.nx;
  d.otau = (int64_t)a * s.n_tau;
  d.ost = (int64_t)a * s.N * s.n_feet;
  d.omu = a;
  d.ox = (int64_t)a * (s.N + 1) * s.nx;
  d.ou = (int64_t)a * s.N * s.nu;
  d.our = d.ou;
  d.oz = (int64_t)a * s.N * m;
  d.oy = d.oz;
  d.ows = 0;
  d.ofw = (int64_t)a * fws_per_agent;
  out[a] = d;
  list[a] = a;
}

}  // namespace

extern "C" mpc_status mpc_solve_noalloc(const mpc_plan_desc* desc, const mpc_problem_batch* b,
                                        const mpc_solution* io, void* stream) {
  if (!desc || !b || !io) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  if (desc->n_agents <= 0 || !desc->shapes)
    return api_fail(MPC_ERR_INVALID_ARG, "n_agents must be > 0 with a shapes array");
  if (desc->precision != MPC_FP32)
    return api_fail(MPC_ERR_INVALID_ARG, "the no-allocation solve is FP32 only");
  if (desc->admm_iters <= 0) return api_fail(MPC_ERR_INVALID_ARG, "admm_iters must be > 0");
  if (desc->scaling_iters != 0 || desc->rho_interval != 0 || desc->joint_limits != 0 ||
      desc->no_slip != 0 || desc->inner_solve != 0 || desc->riccati_scan != 0 || b->x_lo ||
      b->J_foot || b->x_hi)
    return api_fail(MPC_ERR_INVALID_ARG,
                    "the no-allocation solve runs the serial Riccati solve without scaling, joint limits or no-slip rows and with a fixed rho");
  if (!(desc->rho > 0) || !(desc->sigma >= 0) || !(desc->alpha > 0 && desc->alpha < 2) ||
      !(desc->rho_eq_scale > 0) || !(desc->rho_min > 0))
    return api_fail(MPC_ERR_INVALID_ARG, "solver constants out of range");
  if (desc->device < 0 || desc->device >= kMaxDevices)
    return api_fail(MPC_ERR_INVALID_ARG, "device ordinal out of range");
  const mpc_shape s = desc->shapes[0];
  for (int a = 1; a < desc->n_agents; ++a) {
    const mpc_shape& t = desc->shapes[a];
    if (memcmp(&t, &s, sizeof s) != 0)
      return api_fail(MPC_ERR_UNSUPPORTED_SHAPE, "the no-allocation solve needs one shape for every agent");
  }
  if (s.N < 1 || s.nx < 1 || s.nu < 1 || s.n_feet < 0 || s.n_tau < 0 ||
      (s.foot_dim != 3 && s.foot_dim != 6) || s.nu != s.n_tau + s.n_feet * s.foot_dim ||
      !fused_supported(s.N, s.nx, s.nu, s.n_feet))
    return api_fail(MPC_ERR_UNSUPPORTED_SHAPE,
                    "the no-allocation solve runs the register-resident kernels: (nx, nu) = (48, 30) "
                    "or (36, 24), N <= 20");
  if (!b->A || !b->B || !b->c || !b->q_diag || !b->r_diag || !b->x_ref || !b->x0 || !b->mu ||
      (s.n_tau > 0 && !b->tau_max) || (s.n_feet > 0 && !b->stance))
    return api_fail(MPC_ERR_INVALID_ARG, "null input pointer in batch");
  if (b->warm_start != 0 && b->warm_start != 1)
    return api_fail(MPC_ERR_INVALID_ARG, "warm_start must be 0 or 1");
  if (!io->x || !io->u || !io->z || !io->y || !io->objective || !io->residuals || !io->status)
    return api_fail(MPC_ERR_INVALID_ARG,
                    "the no-allocation solve keeps its iterate in the caller's x, u, z, y, objective, "
                    "residuals and status buffers: none may be NULL");

  const int n = desc->n_agents;
  const int64_t per_agent = (int64_t)fused_agent_floats(s.N, s.nx, s.nu);
  const size_t off_list = align256(sizeof(AgentDesc) * (size_t)n);
  const size_t off_fws = align256(off_list + sizeof(int32_t) * (size_t)n);
  const size_t need = off_fws + sizeof(float) * (size_t)per_agent * (size_t)n;
  if (need > (size_t)MPC_NOALLOC_SCRATCH_BYTES) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "batch needs %zu bytes of scratch; the no-allocation solve has %zu (at most %d agents "
             "of this shape)",
             need, (size_t)MPC_NOALLOC_SCRATCH_BYTES,
             (int)(((size_t)MPC_NOALLOC_SCRATCH_BYTES - 512) /
                   (sizeof(AgentDesc) + sizeof(int32_t) + sizeof(float) * (size_t)per_agent)));
    return api_fail(MPC_ERR_UNSUPPORTED_SHAPE, buf);
  }

  MPC_HIP_TRY(hipSetDevice(desc->device));
  void* base = nullptr;
  mpc_status ps = scratch_ptr(desc->device, &base);
  if (ps != MPC_OK) return ps;
  hipStream_t st = (hipStream_t)stream;
  AgentDesc* d_desc = (AgentDesc*)base;
  int32_t* d_list = (int32_t*)((char*)base + off_list);
  float* d_fws = (float*)((char*)base + off_fws);

  hipLaunchKernelGGL(k_uniform_desc, dim3((n + 255) / 256), dim3(256), 0, st, s, n, per_agent,
                     d_desc, d_list);
  MPC_HIP_TRY(hipGetLastError());

  Inputs<float> in;
  in.A = (const float*)b->A;
  in.B = (const float*)b->B;
  in.c = (const float*)b->c;
  in.q = (const float*)b->q_diag;
  in.r = (const float*)b->r_diag;
  in.xr = (const float*)b->x_ref;
  in.x0 = (const float*)b->x0;
  in.tau = (const float*)b->tau_max;
  in.mu = (const float*)b->mu;
  in.st = b->stance;
  in.uref = (const float*)b->u_ref;
  State<float> sv;
  sv.x = (float*)io->x;
  sv.u = (float*)io->u;
  sv.z = (float*)io->z;
  sv.y = (float*)io->y;
  sv.obj = (float*)io->objective;
  sv.res = io->residuals;
  sv.status = io->status;
  const SolverConsts sc{desc->rho, desc->sigma, desc->alpha, desc->rho_eq_scale, desc->rho_min};
  // factor (writes every agent's status) and iterations; every operator slot
  // the iterations read is written by the factor first, so nothing is cleared
  MPC_HIP_TRY(fused_solve_f32(d_desc, d_list, n, s.N, s.nx, s.nu, s.n_feet, in, sc,
                              desc->admm_iters, b->warm_start, sv, d_fws, st, 3));
  const size_t lds_res = generic_residual_lds(s.N, s.nx, s.nu, sizeof(float));
  MPC_HIP_TRY(generic_set_lds_limits(0, 0, lds_res));
  MPC_HIP_TRY(launch_residual<float>(d_desc, d_list, n, in, sc, sv, lds_res, st));
  if (io->u0)
    MPC_HIP_TRY(hipMemcpy2DAsync(io->u0, sizeof(float) * s.nu, io->u, sizeof(float) * s.N * s.nu,
                                 sizeof(float) * s.nu, n, hipMemcpyDeviceToDevice, st));
  return MPC_OK;
}
