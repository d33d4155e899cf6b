// Host side of the C ABI declared in include/mpc.h: plan creation and
// validation, device workspace, kernel dispatch, solution export, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mpc.h"
#include "fused.h"
#include "host_api.h"
#include "mpc_internal.h"
#include "scaling.h"

using namespace mpc;

namespace mpc {
namespace {
thread_local std::string g_err;
}  // namespace

mpc_status api_fail(mpc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace mpc

namespace {

mpc_status fail(mpc_status s, const std::string& msg) { return api_fail(s, msg); }

#define HIP_TRY(expr) MPC_HIP_TRY(expr)

constexpr int kPhases = 3;
constexpr int kMaxAuxStreams = 3;  // plus the caller's stream: four hardware queues

// A launch group: agents of one shape class (and, for the register-resident
// kernels, one horizon) solved by one kernel family with one launch shape.
struct Group {
  int family = 1;          // 1 generic, 2 register-resident, 4 mixed precision
  bool fused_ok = false;   // register-resident kernels have an instantiation for it
  int N = 0, nx = 0, nu = 0, n_feet = 0;  // N: largest horizon in the group
  int nc = 0;              // no-slip rows per state (plans with them)
  int count = 0;
  int64_t list_off = 0;    // agents d_list[list_off .. list_off + count)
  int gthreads = 256;      // generic workgroup size
  size_t lds_factor = 0, lds_admm = 0;
  int fthreads = 0;        // register-resident iteration-kernel workgroup size
  size_t flds = 0;
  double work = 0;         // relative cost used to order launches
  double est = 0;          // cost estimate for the queue assignment (ms once autotuned)
  int queue = 0;           // 0: the caller's stream, k > 0: aux stream k - 1
  bool persistent = false; // register-resident family: one persistent launch, every horizon
  int counter = -1;        // its work-queue counter: d_counters[counter]
  int64_t scan_off = 0;    // parallel-in-time factor: its element buffers at d_scan + scan_off
};

// Longest group first onto the least-loaded of nq queues (each queue runs its
// groups in order, the queues run concurrently).
void assign_queues(std::vector<Group>& groups, int nq) {
  std::vector<size_t> order(groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return groups[x].est > groups[y].est; });
  std::vector<double> load(std::max(nq, 1), 0.0);
  for (size_t i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    groups[i].queue = k;
    load[k] += groups[i].est;
  }
}

// u_0 of every agent into a packed [sum nu] buffer (agent a's block at
// u0off[a]), for batches whose u blocks are not evenly strided.
template <typename T>
__global__ void __launch_bounds__(64)
k_gather_u0_packed(const AgentDesc* __restrict__ desc, const int64_t* __restrict__ u0off, int n,
                   const T* __restrict__ u, T* __restrict__ u0) {
  const int a = blockIdx.x;
  if (a >= n) return;
  const int64_t src = desc[a].ou, dst = u0off[a];
  const int nu = desc[a].nu;
  for (int j = threadIdx.x; j < nu; j += blockDim.x) u0[dst + j] = u[src + j];
}

}  // namespace

struct mpc_plan_s {
  mpc_plan_desc desc{};
  std::vector<mpc_shape> shapes;
  std::vector<AgentDesc> hdesc;
  int n = 0;
  bool fp64 = false;
  size_t esz = 4;
  int kernel = 1;
  int maxN = 0, maxnx = 0, maxnu = 0, maxm = 0;
  int64_t nX = 0, nU = 0, nZ = 0, nWS = 0;
  int64_t nC = 0;  // sum of N nx (the layout of c)
  AgentDesc* d_desc = nullptr;
  int64_t* d_u0off = nullptr;  // packed u_0 offset of every agent
  bool uniform_u = true;       // every agent has the same N and nu
  void* d_ws = nullptr;
  void *d_x = nullptr, *d_u = nullptr, *d_z = nullptr, *d_y = nullptr, *d_obj = nullptr;
  double* d_res = nullptr;
  int32_t* d_status = nullptr;
  // scaling (Ruiz) and adaptive rho
  bool scaled = false, adaptive = false;
  void* d_sbuf = nullptr;          // the scaled problem data
  int64_t s_off[9] = {};           // element offsets of A, B, c, q, r, x_ref, x0, tau, mu in d_sbuf
  double* d_scale = nullptr;       // [n][kScaleStride]
  double* d_rho = nullptr;         // [n]
  double* d_rho_hist = nullptr;    // [n][n_seg]: the rho of every segment
  // joint limits
  bool limits = false;
  void *d_zx = nullptr, *d_yx = nullptr;  // [sum N nx]: the state rows' (z_x, y_x)
  int64_t nZX = 0;
  // paper-form inner solve (finite rho_eq, KKT factored by LDL^T)
  bool kkt = false;
  void *d_zd = nullptr, *d_yd = nullptr;  // [sum N nx]: the dynamics rows' (z, y)
  size_t lds_kkt_factor = 0, lds_kkt_admm = 0;
  // no-slip rows
  bool contacts = false;
  void *d_zc = nullptr, *d_yc = nullptr;  // [sum N n_feet foot_dim]: the rows' (z_c, y_c)
  int64_t nZC = 0, maxnc = 0;
  int n_seg = 1;
  bool solved = false;
  bool kkt_state = false;  // x, zd, yd hold an iterate (KKT inner solve)
  size_t lds_factor = 0, lds_admm = 0, lds_res = 0;
  // launch groups
  std::vector<Group> groups;
  std::vector<int32_t> hlist;
  int32_t* d_list = nullptr;
  int* d_counters = nullptr;  // one work-queue counter per persistent group
  bool scan = false;          // generic factor by the parallel-in-time scan
  double* d_scan = nullptr;   // its element buffers (Group::scan_off)
  float* d_fws = nullptr;
  int64_t nFWS = 0;
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  // captured step
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool capturing = false;
  // timing
  bool timing = false;
  hipStream_t last_stream = nullptr;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[kPhases] = {0, 0, 0};
  int64_t launches[kPhases] = {0, 0, 0};
};

static mpc_status validate_shape(const mpc_shape& s, int idx) {
  char buf[256];
  if (s.N < 1 || s.N > 64 || s.nx < 1 || s.nx > 64 || s.nu < 1 || s.nu > 32 || s.n_feet < 0 ||
      s.n_feet > 8 || s.n_tau < 0 || (s.foot_dim != 3 && s.foot_dim != 6) ||
      s.nu != s.n_tau + s.n_feet * s.foot_dim) {
    snprintf(buf, sizeof buf,
             "agent %d: unsupported shape (N=%d nx=%d nu=%d n_tau=%d n_feet=%d foot_dim=%d)", idx,
             s.N, s.nx, s.nu, s.n_tau, s.n_feet, s.foot_dim);
    return fail(MPC_ERR_UNSUPPORTED_SHAPE, buf);
  }
  return MPC_OK;
}

extern "C" void mpc_plan_desc_default(mpc_plan_desc* d) {
  if (!d) return;
  memset(d, 0, sizeof(*d));
  d->precision = MPC_FP32;
  d->admm_iters = 50;
  d->rho = 0.1;
  d->sigma = 1e-6;
  d->alpha = 1.6;
  d->rho_eq_scale = 1e3;
  d->rho_min = 1e-6;
  d->max_refine_sweeps = 3;
  d->refine_tol = 1e-6;
  d->device = 0;
  d->kernel = 0;
  d->scaling_iters = 0;
  d->rho_interval = 0;
  d->rho_tolerance = 5.0;
  d->joint_limits = 0;
  d->no_slip = 0;
  d->inner_solve = 0;
  d->riccati_scan = 0;
}

extern "C" const char* mpc_last_error(void) { return mpc::g_err.c_str(); }
extern "C" const char* mpc_version(void) { return "mpc-mi355x 0.1.0 (gfx950)"; }

static void free_plan(mpc_plan_s* p) {
  if (!p) return;
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  for (auto st : p->aux) hipStreamDestroy(st);
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  for (auto e : p->ev_join) hipEventDestroy(e);
  hipFree(p->d_desc);
  hipFree(p->d_u0off);
  hipFree(p->d_list);
  hipFree(p->d_counters);
  hipFree(p->d_scan);
  hipFree(p->d_fws);
  hipFree(p->d_ws);
  hipFree(p->d_x);
  hipFree(p->d_u);
  hipFree(p->d_z);
  hipFree(p->d_y);
  hipFree(p->d_obj);
  hipFree(p->d_res);
  hipFree(p->d_status);
  hipFree(p->d_sbuf);
  hipFree(p->d_scale);
  hipFree(p->d_rho);
  hipFree(p->d_rho_hist);
  hipFree(p->d_zx);
  hipFree(p->d_yx);
  hipFree(p->d_zc);
  hipFree(p->d_yc);
  hipFree(p->d_zd);
  hipFree(p->d_yd);
  for (auto e : p->ev_pool) hipEventDestroy(e);
  for (auto& pe : p->pending) {
    hipEventDestroy(pe.second.first);
    hipEventDestroy(pe.second.second);
  }
  delete p;
}

extern "C" mpc_status mpc_plan_create(const mpc_plan_desc* desc, mpc_plan_t* out) {
  if (!desc || !out) return fail(MPC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (desc->n_agents <= 0 || !desc->shapes) return fail(MPC_ERR_INVALID_ARG, "n_agents must be > 0 with a shapes array");
  if (desc->precision < MPC_FP64 || desc->precision > MPC_FP32_MFMA)
    return fail(MPC_ERR_INVALID_ARG, "unknown precision");
  if (desc->admm_iters <= 0) return fail(MPC_ERR_INVALID_ARG, "admm_iters must be > 0");
  if (!(desc->rho > 0) || !(desc->sigma >= 0) || !(desc->alpha > 0 && desc->alpha < 2) ||
      !(desc->rho_eq_scale > 0) || !(desc->rho_min > 0) || !std::isfinite(desc->rho) ||
      !std::isfinite(desc->sigma) || !std::isfinite(desc->rho_eq_scale) || !std::isfinite(desc->rho_min))
    return fail(MPC_ERR_INVALID_ARG, "solver constants out of range (rho>0, sigma>=0, 0<alpha<2, rho_eq_scale>0, rho_min>0)");
  if (desc->kernel < 0 || desc->kernel > 3) return fail(MPC_ERR_INVALID_ARG, "unknown kernel selector");
  if (desc->max_refine_sweeps < 0 || desc->max_refine_sweeps > 16 || !(desc->refine_tol >= 0) ||
      !std::isfinite(desc->refine_tol))
    return fail(MPC_ERR_INVALID_ARG, "max_refine_sweeps must be in 0..16 and refine_tol >= 0");
  if (desc->scaling_iters < 0 || desc->scaling_iters > 100 || desc->rho_interval < 0 ||
      (desc->rho_interval > 0 && !(desc->rho_tolerance >= 1.0 && std::isfinite(desc->rho_tolerance))))
    return fail(MPC_ERR_INVALID_ARG,
                "scaling_iters must be in 0..100, rho_interval >= 0 and rho_tolerance >= 1");
  if (desc->joint_limits != 0 && desc->joint_limits != 1)
    return fail(MPC_ERR_INVALID_ARG, "joint_limits must be 0 or 1");
  if (desc->joint_limits &&
      (refine_precision(desc->precision) ||
       desc->scaling_iters > 0 || desc->kernel == 2))
    return fail(MPC_ERR_INVALID_ARG,
                "joint limits run on the generic kernels in FP64 or FP32, without scaling");
  if (desc->no_slip != 0 && desc->no_slip != 1) return fail(MPC_ERR_INVALID_ARG, "no_slip must be 0 or 1");
  if (desc->no_slip &&
      (refine_precision(desc->precision) ||
       desc->scaling_iters > 0 || desc->kernel == 3))
    return fail(MPC_ERR_INVALID_ARG,
                "no-slip rows run on the generic or register-resident kernels in FP64 or FP32, "
                "without scaling or the persistent launch");
  if (desc->inner_solve != 0 && desc->inner_solve != 1)
    return fail(MPC_ERR_INVALID_ARG, "inner_solve must be 0 or 1");
  if (desc->precision == MPC_FP32_MFMA &&
      (desc->kernel == 1 || desc->joint_limits || desc->no_slip || desc->inner_solve ||
       desc->riccati_scan))
    return fail(MPC_ERR_INVALID_ARG,
                "MPC_FP32_MFMA runs the register-resident kernels: not with kernel = 1, joint "
                "limits, no-slip rows, the KKT inner solve or the parallel-in-time factor");
  if (desc->riccati_scan != 0 && desc->riccati_scan != 1)
    return fail(MPC_ERR_INVALID_ARG, "riccati_scan must be 0 or 1");
  if (desc->riccati_scan &&
      (refine_precision(desc->precision) || desc->inner_solve ||
       desc->kernel == 2 || desc->kernel == 3))
    return fail(MPC_ERR_INVALID_ARG,
                "the parallel-in-time factor runs on the generic kernels in FP64 or FP32, "
                "not with the KKT inner solve");
  if (desc->inner_solve &&
      (refine_precision(desc->precision) ||
       desc->scaling_iters > 0 || desc->rho_interval > 0 || desc->kernel == 2 ||
       desc->joint_limits || desc->no_slip))
    return fail(MPC_ERR_INVALID_ARG,
                "the KKT inner solve runs on its own kernels in FP64 or FP32, with a fixed rho and "
                "without scaling, joint limits or no-slip rows");
  for (int a = 0; a < desc->n_agents; ++a) {
    mpc_status vs = validate_shape(desc->shapes[a], a);
    if (vs != MPC_OK) return vs;
    if (desc->riccati_scan && desc->shapes[a].nx > 48)
      return fail(MPC_ERR_UNSUPPORTED_SHAPE,
                  "the parallel-in-time factor keeps a combine's six nx x nx blocks in LDS: nx <= 48");
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (desc->device < 0 || desc->device >= ndev) return fail(MPC_ERR_INVALID_ARG, "device ordinal out of range");

  auto* p = new mpc_plan_s();
  p->desc = *desc;
  p->n = desc->n_agents;
  p->shapes.assign(desc->shapes, desc->shapes + desc->n_agents);
  p->desc.shapes = nullptr;
  p->fp64 = desc->precision == MPC_FP64;
  p->esz = p->fp64 ? 8 : 4;
  p->limits = desc->joint_limits != 0;
  p->contacts = desc->no_slip != 0;
  p->kkt = desc->inner_solve != 0;
  p->scan = desc->riccati_scan != 0;

  p->hdesc.resize(p->n);
  AgentDesc cur{};
  int64_t oA = 0, oB = 0, oc = 0, oq = 0, orr = 0, oxr = 0, ox0 = 0, otau = 0, ost = 0, ox = 0,
          ou = 0, oz = 0, ows = 0, oJ = 0, ozc = 0;
  for (int a = 0; a < p->n; ++a) {
    const mpc_shape& s = p->shapes[a];
    cur.N = s.N;
    cur.nx = s.nx;
    cur.nu = s.nu;
    cur.n_tau = s.n_tau;
    cur.n_feet = s.n_feet;
    cur.foot_dim = s.foot_dim;
    cur.m = s.nu + 4 * s.n_feet;
    cur.oA = oA; cur.oB = oB; cur.oc = oc; cur.oq = oq; cur.orr = orr; cur.oxr = oxr;
    cur.ox0 = ox0; cur.otau = otau; cur.ost = ost; cur.ox = ox; cur.ou = ou; cur.oz = oz;
    cur.ows = ows;
    cur.ofw = -1;
    cur.oy = oz;
    cur.omu = a;
    cur.our = ou;
    cur.flags = 0;
    cur.oJ = oJ;
    cur.ozc = ozc;
    p->hdesc[a] = cur;
    oJ += (int64_t)s.n_feet * s.foot_dim * s.nx;
    ozc += (int64_t)s.N * s.n_feet * s.foot_dim;
    p->maxnc = std::max<int64_t>(p->maxnc, (int64_t)s.n_feet * s.foot_dim);
    oA += (int64_t)s.N * s.nx * s.nx;
    oB += (int64_t)s.N * s.nx * s.nu;
    oc += (int64_t)s.N * s.nx;
    oq += s.nx;
    orr += s.nu;
    oxr += (int64_t)(s.N + 1) * s.nx;
    ox0 += s.nx;
    otau += s.n_tau;
    ost += (int64_t)s.N * s.n_feet;
    ox += (int64_t)(s.N + 1) * s.nx;
    ou += (int64_t)s.N * s.nu;
    oz += (int64_t)s.N * cur.m;
    ows += p->kkt ? kkt_ws_elems(s.N, s.nx, s.nu) : generic_ws_elems(s.N, s.nx, s.nu, cur.m);
    if (p->kkt) {
      p->lds_kkt_factor = std::max(p->lds_kkt_factor, kkt_factor_lds(s.nx, s.nu, cur.m));
      p->lds_kkt_admm = std::max(p->lds_kkt_admm, kkt_admm_lds(s.N, s.nx, s.nu, cur.m));
    }
    p->maxN = std::max(p->maxN, s.N);
    p->maxnx = std::max(p->maxnx, s.nx);
    p->maxnu = std::max(p->maxnu, s.nu);
    p->maxm = std::max(p->maxm, cur.m);
  }
  p->nX = ox;
  p->nU = ou;
  p->nZ = oz;
  p->nWS = ows;
  p->nC = oc;
  p->lds_factor = generic_factor_lds(p->maxnx, p->maxnu, p->esz);
  p->lds_admm = generic_admm_lds(p->maxN, p->maxnx, p->maxnu, p->maxm, p->esz, p->limits,
                                 p->contacts ? (int)p->maxnc : 0);
  p->lds_res = generic_residual_lds(p->maxN, p->maxnx, p->maxnu, p->esz);

  // Launch groups.  FP32 agents whose shape has a register-resident
  // instantiation are grouped per (shape class, horizon) and take those
  // kernels; every other agent is grouped per shape class and takes the
  // generic kernels, sized for the group's longest horizon.
  const bool mixed = refine_precision(desc->precision);
  int n_counters = 0;
  {
    std::map<std::tuple<int, int, int, int, int, int, int>, std::vector<int32_t>> buckets;
    for (int a = 0; a < p->n; ++a) {
      const mpc_shape& s = p->shapes[a];
      // no-slip rows: the register-resident body when asked for (kernel = 2),
      // since its FP32 chains carry the stiff rows' large duals (the generic
      // kernels accumulate in FP64)
      const int nca = p->contacts ? s.n_feet * s.foot_dim : 0;
      const bool fok = (desc->precision == MPC_FP32 || desc->precision == MPC_FP32_MFMA) &&
                       !p->limits && !p->kkt && !(nca && desc->kernel != 2) &&
                       fused_supported(s.N, s.nx, s.nu, s.n_feet, nca);
      if ((desc->kernel == 2 || desc->kernel == 3 || desc->precision == MPC_FP32_MFMA) && !fok) {
        delete p;
        return fail(MPC_ERR_UNSUPPORTED_SHAPE,
                    "register-resident kernels requested for an agent they do not support");
      }
      if (mixed && !mixed_supported(s.nx, s.nu)) {
        delete p;
        return fail(MPC_ERR_UNSUPPORTED_SHAPE,
                    "mixed precision is built for (nx, nu) = (48, 30) and (36, 24) only");
      }
      const bool use_fused = fok && desc->kernel != 1 && !mixed && !p->scan;
      const int fam = mixed ? 4 : use_fused ? 2 : 1;
      buckets[std::make_tuple(fam, s.nx, s.nu, s.n_tau, s.n_feet, s.foot_dim,
                              use_fused && desc->kernel != 3 ? fused_bucket(s.N) : 0)]
          .push_back(a);
    }
    for (auto& kv : buckets) {
      Group g;
      g.family = std::get<0>(kv.first);
      g.fused_ok = g.family == 2;
      std::vector<int32_t>& ag = kv.second;
      // longest horizon first so the tail of a generic launch is short
      std::stable_sort(ag.begin(), ag.end(),
                       [&](int32_t x, int32_t y) { return p->shapes[x].N > p->shapes[y].N; });
      const mpc_shape& s0 = p->shapes[ag[0]];
      g.N = s0.N;
      g.nx = s0.nx;
      g.nu = s0.nu;
      g.n_feet = s0.n_feet;
      g.nc = s0.n_feet * s0.foot_dim;
      g.count = (int)ag.size();
      g.list_off = (int64_t)p->hlist.size();
      const int m = s0.nu + 4 * s0.n_feet;
      g.lds_factor = generic_factor_lds(s0.nx, s0.nu, p->esz);
      g.lds_admm = generic_admm_lds(g.N, s0.nx, s0.nu, m, p->esz, p->limits,
                                    p->contacts ? s0.n_feet * s0.foot_dim : 0);
      if (g.fused_ok)
        fused_launch_shape(g.N, g.nx, g.nu, g.n_feet, &g.fthreads, &g.flds,
                           p->contacts ? s0.n_feet * s0.foot_dim : 0);
      if (g.fused_ok && desc->kernel == 3) {
        g.persistent = true;
        g.counter = n_counters++;
        fused_persistent_shape(g.N, g.nx, g.nu, g.n_feet, &g.fthreads, &g.flds);
      }
      for (int32_t a : ag) g.work += (double)p->shapes[a].N * (s0.nx + s0.nu) * (s0.nx + s0.nu);
      g.est = g.work;
      p->hlist.insert(p->hlist.end(), ag.begin(), ag.end());
      p->groups.push_back(g);
    }
    std::stable_sort(p->groups.begin(), p->groups.end(),
                     [](const Group& x, const Group& y) { return x.work > y.work; });
  }
  // register-resident workspace for every agent of a group that may use it
  for (const Group& g : p->groups) {
    if (!g.fused_ok) continue;
    for (int i = 0; i < g.count; ++i) {
      const int32_t a = p->hlist[g.list_off + i];
      p->hdesc[a].ofw = p->nFWS;
      p->nFWS += (int64_t)fused_agent_floats(p->shapes[a].N, g.nx, g.nu);
    }
  }
  p->kernel = 0;
  for (const Group& g : p->groups) p->kernel |= g.family;

  hipError_t e = hipSetDevice(desc->device);
  if (e != hipSuccess) {
    delete p;
    return fail(MPC_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  int lds_max = 0;
  hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, desc->device);
  if ((int64_t)p->lds_factor > lds_max || (int64_t)p->lds_admm > lds_max ||
      (int64_t)p->lds_kkt_factor > lds_max || (int64_t)p->lds_kkt_admm > lds_max) {
    delete p;
    return fail(MPC_ERR_UNSUPPORTED_SHAPE, "shapes need more LDS than the device offers");
  }
  e = generic_set_lds_limits(p->lds_factor, p->lds_admm, p->lds_res);
  if (e == hipSuccess && p->kkt) e = kkt_set_lds_limits(p->lds_kkt_factor, p->lds_kkt_admm);
  if (e == hipSuccess && p->scan) e = scan_set_limits();
  if (e == hipSuccess && !p->fp64) e = fused_set_limits();
  if (e != hipSuccess) {
    delete p;
    return fail(MPC_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  auto alloc = [&](void** ptr, size_t bytes) -> hipError_t {
    return hipMalloc(ptr, bytes ? bytes : 16);
  };
  std::vector<int64_t> u0off(p->n);
  for (int a = 0, off = 0; a < p->n; ++a) {
    u0off[a] = off;
    off += p->shapes[a].nu;
    p->uniform_u &= p->shapes[a].N == p->shapes[0].N && p->shapes[a].nu == p->shapes[0].nu;
  }
  hipError_t errs[13] = {
      alloc((void**)&p->d_desc, sizeof(AgentDesc) * p->n),
      alloc((void**)&p->d_u0off, sizeof(int64_t) * p->n),
      alloc((void**)&p->d_list, sizeof(int32_t) * p->hlist.size()),
      alloc((void**)&p->d_counters, sizeof(int) * (size_t)std::max(n_counters, 1)),
      alloc((void**)&p->d_fws, sizeof(float) * (size_t)p->nFWS),
      alloc(&p->d_ws, p->esz * (size_t)p->nWS),
      alloc(&p->d_x, p->esz * (size_t)p->nX),
      alloc(&p->d_u, p->esz * (size_t)p->nU),
      alloc(&p->d_z, p->esz * (size_t)p->nZ),
      alloc(&p->d_y, p->esz * (size_t)p->nZ),
      alloc(&p->d_obj, p->esz * (size_t)p->n),
      alloc((void**)&p->d_res, sizeof(double) * 4 * (size_t)p->n),
      alloc((void**)&p->d_status, sizeof(int32_t) * (size_t)p->n)};
  for (hipError_t ee : errs) {
    if (ee != hipSuccess) {
      mpc_status st = fail(ee == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,
                           std::string("hipMalloc: ") + hipGetErrorString(ee));
      free_plan(p);
      return st;
    }
  }
  p->scaled = desc->scaling_iters > 0;
  p->adaptive = desc->rho_interval > 0;
  {
    hipError_t se = hipSuccess;
    if (p->scaled) {
      const int64_t sizes[9] = {oA, oB, oc, oq, orr, oxr, ox0, otau, (int64_t)p->n};
      int64_t tot = 0;
      for (int i = 0; i < 9; ++i) {
        p->s_off[i] = tot;
        tot += (sizes[i] + 63) / 64 * 64;  // 256-byte aligned parts
      }
      se = alloc(&p->d_sbuf, p->esz * (size_t)tot);
      if (se == hipSuccess) se = alloc((void**)&p->d_scale, sizeof(double) * kScaleStride * (size_t)p->n);
    }
    if (p->adaptive) p->n_seg = (desc->admm_iters + desc->rho_interval - 1) / desc->rho_interval;
    if (se == hipSuccess && p->adaptive) se = alloc((void**)&p->d_rho, sizeof(double) * (size_t)p->n);
    if (se == hipSuccess && p->adaptive)
      se = alloc((void**)&p->d_rho_hist, sizeof(double) * (size_t)p->n * p->n_seg);
    if (p->limits) {
      p->nZX = oc;  // N nx per agent, the layout of c
      if (se == hipSuccess) se = alloc(&p->d_zx, p->esz * (size_t)p->nZX);
      if (se == hipSuccess) se = alloc(&p->d_yx, p->esz * (size_t)p->nZX);
    }
    if (p->kkt) {
      if (se == hipSuccess) se = alloc(&p->d_zd, p->esz * (size_t)oc);
      if (se == hipSuccess) se = alloc(&p->d_yd, p->esz * (size_t)oc);
    }
    if (p->scan) {
      // two element buffers per group, side by side
      size_t off = 0;
      for (Group& g : p->groups) {
        g.scan_off = (int64_t)(off / sizeof(double));
        off += 2 * scan_elements_bytes(g.count, g.N, g.nx);
      }
      if (se == hipSuccess) se = alloc((void**)&p->d_scan, std::max<size_t>(off, 16));
    }
    if (p->contacts) {
      p->nZC = ozc;
      if (se == hipSuccess) se = alloc(&p->d_zc, p->esz * (size_t)std::max<int64_t>(p->nZC, 1));
      if (se == hipSuccess) se = alloc(&p->d_yc, p->esz * (size_t)std::max<int64_t>(p->nZC, 1));
    }
    if (se != hipSuccess) {
      mpc_status st = fail(se == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,
                           std::string("hipMalloc: ") + hipGetErrorString(se));
      free_plan(p);
      return st;
    }
  }
  e = hipMemcpy(p->d_desc, p->hdesc.data(), sizeof(AgentDesc) * p->n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_u0off, u0off.data(), sizeof(int64_t) * p->n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_list, p->hlist.data(), sizeof(int32_t) * p->hlist.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->d_status, 0, sizeof(int32_t) * p->n);
  // concurrent streams for the launch groups (default priority)
  const int naux = std::min<int>((int)p->groups.size() - 1, kMaxAuxStreams);
  if (e == hipSuccess && naux > 0) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  for (int i = 0; i < naux && e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) p->aux.push_back(st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) p->ev_join.push_back(ev);
  }
  assign_queues(p->groups, 1 + (int)p->aux.size());
  if (e != hipSuccess) {
    free_plan(p);
    return fail(MPC_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *out = p;
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_destroy(mpc_plan_t p) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  hipSetDevice(p->desc.device);
  hipDeviceSynchronize();
  free_plan(p);
  return MPC_OK;
}

static mpc_status check_batch(mpc_plan_s* p, const mpc_problem_batch* b) {
  if (!b) return fail(MPC_ERR_INVALID_ARG, "null batch");
  if (!b->A || !b->B || !b->c || !b->q_diag || !b->r_diag || !b->x_ref || !b->x0 || !b->mu)
    return fail(MPC_ERR_INVALID_ARG, "null input pointer in batch");
  // tau_max and stance may be NULL only when no agent has torques / feet
  bool any_tau = false, any_feet = false;
  for (const auto& s : p->shapes) {
    any_tau |= s.n_tau > 0;
    any_feet |= s.n_feet > 0;
  }
  if (any_tau && !b->tau_max) return fail(MPC_ERR_INVALID_ARG, "null tau_max");
  if (any_feet && !b->stance) return fail(MPC_ERR_INVALID_ARG, "null stance");
  if (b->warm_start != 0 && b->warm_start != 1) return fail(MPC_ERR_INVALID_ARG, "warm_start must be 0 or 1");
  if (b->warm_start && !p->solved)
    return fail(MPC_ERR_INVALID_ARG, "warm_start requested before any solve or warm state");
  if (b->warm_start && p->kkt && !p->kkt_state)
    return fail(MPC_ERR_INVALID_ARG,
                "warm_start of the KKT inner solve needs a previous solve or mpc_set_warm_kkt");
  if (p->scaled && b->u_ref)
    return fail(MPC_ERR_INVALID_ARG, "an input reference is not supported with scaling");
  if (p->limits != (b->x_lo != nullptr) || (b->x_lo == nullptr) != (b->x_hi == nullptr))
    return fail(MPC_ERR_INVALID_ARG,
                p->limits ? "this plan solves with joint limits: x_lo and x_hi are required"
                          : "x_lo / x_hi given to a plan created without joint limits");
  if (p->contacts != (b->J_foot != nullptr))
    return fail(MPC_ERR_INVALID_ARG,
                p->contacts ? "this plan solves with no-slip rows: J_foot is required"
                            : "J_foot given to a plan created without no-slip rows");
  return MPC_OK;
}

// The batch the iterations run on: the plan's scaled copy of the caller's data
// (stance from the caller) when the plan equilibrates, else the caller's.
static mpc_problem_batch solver_batch(mpc_plan_s* p, const mpc_problem_batch* b) {
  mpc_problem_batch sb = *b;
  if (!p->scaled) return sb;
  char* base = (char*)p->d_sbuf;
  const void** f[9] = {&sb.A, &sb.B, &sb.c, &sb.q_diag, &sb.r_diag, &sb.x_ref, &sb.x0, &sb.tau_max, &sb.mu};
  for (int i = 0; i < 9; ++i) *f[i] = base + p->s_off[i] * (int64_t)p->esz;
  sb.u_ref = nullptr;
  return sb;
}

template <typename T>
static ScaledInputs<T> scaled_out(mpc_plan_s* p) {
  T* base = (T*)p->d_sbuf;
  ScaledInputs<T> o;
  T** f[9] = {&o.A, &o.B, &o.c, &o.q, &o.r, &o.xr, &o.x0, &o.tau, &o.mu};
  for (int i = 0; i < 9; ++i) *f[i] = base + p->s_off[i];
  return o;
}

template <typename T>
static Inputs<T> make_inputs(const mpc_problem_batch* b) {
  Inputs<T> in;
  in.A = (const T*)b->A;
  in.B = (const T*)b->B;
  in.c = (const T*)b->c;
  in.q = (const T*)b->q_diag;
  in.r = (const T*)b->r_diag;
  in.xr = (const T*)b->x_ref;
  in.x0 = (const T*)b->x0;
  in.tau = (const T*)b->tau_max;
  in.mu = (const T*)b->mu;
  in.st = b->stance;
  in.uref = (const T*)b->u_ref;
  in.xlo = (const T*)b->x_lo;
  in.xhi = (const T*)b->x_hi;
  in.J = (const T*)b->J_foot;
  return in;
}

template <typename T>
static State<T> make_state(mpc_plan_s* p) {
  State<T> s;
  s.x = (T*)p->d_x;
  s.u = (T*)p->d_u;
  s.z = (T*)p->d_z;
  s.y = (T*)p->d_y;
  s.obj = (T*)p->d_obj;
  s.res = p->d_res;
  s.status = p->d_status;
  s.zx = (T*)p->d_zx;
  s.yx = (T*)p->d_yx;
  s.zc = (T*)p->d_zc;
  s.yc = (T*)p->d_yc;
  return s;
}

static hipEvent_t get_event(mpc_plan_s* p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// Brackets one launch with events when timing is on.
struct PhaseTimer {
  mpc_plan_s* p;
  int phase;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PhaseTimer(mpc_plan_s* p_, int ph, hipStream_t s_) : p(p_), phase(ph), s(s_) {
    if (p->timing && !p->capturing) {
      e0 = get_event(p);
      e1 = get_event(p);
      hipEventRecord(e0, s);
    }
  }
  ~PhaseTimer() {
    if (e0) {
      hipEventRecord(e1, s);
      p->pending.push_back({phase, {e0, e1}});
    }
  }
};

// Factor and iteration launches of one group on stream s.
template <typename T>
static mpc_status run_group(mpc_plan_s* p, const Group& g, const mpc_problem_batch* b,
                            hipStream_t s, int warm, int iters, bool residual = false) {
  SolverConsts sc{p->desc.rho, p->desc.sigma, p->desc.alpha, p->desc.rho_eq_scale,
                  p->desc.rho_min};
  sc.rho_agent = p->adaptive ? p->d_rho : nullptr;
  const int32_t* list = p->d_list + g.list_off;
  if (g.family == 2) {
    {
      PhaseTimer t(p, 0, s);
      HIP_TRY(fused_solve_f32(p->d_desc, list, g.count, g.N, g.nx, g.nu, g.n_feet,
                              make_inputs<float>(b), sc, iters, warm,
                              make_state<float>(p), p->d_fws, s, 1, nullptr,
                              p->desc.precision == MPC_FP32_MFMA));
    }
    {
      PhaseTimer t(p, 1, s);
      HIP_TRY(fused_solve_f32(p->d_desc, list, g.count, g.N, g.nx, g.nu, g.n_feet,
                              make_inputs<float>(b), sc, iters, warm,
                              make_state<float>(p), p->d_fws, s, 2,
                              g.persistent ? p->d_counters + g.counter : nullptr, false,
                              p->contacts ? g.nc : 0));
    }
  } else if (g.family == 4) {
    {
      PhaseTimer t(p, 0, s);
      HIP_TRY(launch_mixed_factor(p->d_desc, list, g.count, g.nx, g.nu,
                                  refine_product(p->desc.precision),
                                  make_inputs<float>(b), sc, (float*)p->d_ws, p->d_status, s));
    }
    {
      PhaseTimer t(p, 1, s);
      HIP_TRY(launch_generic_admm<float>(p->d_desc, list, g.count, make_inputs<float>(b), sc,
                                         iters, warm, (const float*)p->d_ws,
                                         make_state<float>(p), g.lds_admm, g.gthreads, s,
                                         p->desc.max_refine_sweeps, p->desc.refine_tol));
    }
  } else if (p->kkt) {
    const Inputs<T> in = make_inputs<T>(b);
    {
      PhaseTimer t(p, 0, s);
      HIP_TRY(launch_kkt_factor<T>(p->d_desc, list, g.count, in, sc, (T*)p->d_ws, p->d_status,
                                   kkt_factor_lds(g.nx, g.nu, g.nu + 4 * g.n_feet), s));
    }
    {
      PhaseTimer t(p, 1, s);
      HIP_TRY(launch_kkt_admm<T>(p->d_desc, list, g.count, in, sc, iters, warm,
                                 (const T*)p->d_ws, make_state<T>(p), (T*)p->d_zd, (T*)p->d_yd,
                                 kkt_admm_lds(g.N, g.nx, g.nu, g.nu + 4 * g.n_feet), s));
    }
  } else {
    const Inputs<T> in = make_inputs<T>(b);
    {
      PhaseTimer t(p, 0, s);
      // FP32 plans of the shapes the matrix-core factor is built for take it
      // (FP64 products, generic operator layout) at any horizon, with the
      // joint-limit and no-slip rows' state weights
      if (p->scan) {
        double* E0 = p->d_scan + g.scan_off;
        HIP_TRY(launch_scan_factor<T>(p->d_desc, list, g.count, g.N, g.nx, g.nu, g.nu + 4 * g.n_feet, in, sc,
                                      (T*)p->d_ws, E0, E0 + scan_elements_bytes(g.count, g.N, g.nx) / sizeof(double),
                                      p->d_status, g.lds_factor, s));
      } else if (!p->fp64 && mixed_supported(g.nx, g.nu))
        HIP_TRY(launch_mixed_factor(p->d_desc, list, g.count, g.nx, g.nu, 0, make_inputs<float>(b),
                                    sc, (float*)p->d_ws, p->d_status, s));
      else
        HIP_TRY(launch_generic_factor<T>(p->d_desc, list, g.count, in, sc, (T*)p->d_ws, p->d_status,
                                         g.lds_factor, g.gthreads, s));
    }
    {
      PhaseTimer t(p, 1, s);
      HIP_TRY(launch_generic_admm<T>(p->d_desc, list, g.count, in, sc, iters, warm,
                                     (const T*)p->d_ws, make_state<T>(p), g.lds_admm, g.gthreads,
                                     s));
    }
  }
  if (residual) {
    // the group's KKT residual check on its own queue, so that it overlaps
    // the groups still iterating instead of following the slowest of them
    PhaseTimer t(p, 2, s);
    HIP_TRY(launch_residual<T>(p->d_desc, list, g.count, make_inputs<T>(b), sc, make_state<T>(p),
                               generic_residual_lds(g.N, g.nx, g.nu, p->esz), s));
  }
  return MPC_OK;
}

// Groups run concurrently on the queues assign_queues picked (the caller's
// stream and the aux streams); the aux streams fork from and join back into
// the caller's stream, so the solve stays stream-ordered (and captures into
// one graph).
template <typename T>
static mpc_status run_groups(mpc_plan_s* p, const mpc_problem_batch* b, hipStream_t s, int warm,
                             int iters, bool residual = false) {
  const int ns = 1 + (int)p->aux.size();
  if (ns > 1) {
    HIP_TRY(hipEventRecord(p->ev_fork, s));
    for (hipStream_t a : p->aux) HIP_TRY(hipStreamWaitEvent(a, p->ev_fork, 0));
  }
  for (size_t i = 0; i < p->groups.size(); ++i) {
    const int k = std::min(p->groups[i].queue, ns - 1);
    mpc_status r = run_group<T>(p, p->groups[i], b, k == 0 ? s : p->aux[k - 1], warm, iters, residual);
    if (r != MPC_OK) return r;
  }
  if (ns > 1) {
    for (size_t k = 0; k < p->aux.size(); ++k) {
      HIP_TRY(hipEventRecord(p->ev_join[k], p->aux[k]));
      HIP_TRY(hipStreamWaitEvent(s, p->ev_join[k], 0));
    }
  }
  return MPC_OK;
}

// One solve: (Ruiz scaling,) factor and iterations in segments of rho_interval
// with a rho update between segments (adaptive rho; every segment refactors),
// (unscaling,) then the KKT residual check of the caller's problem.
template <typename T>
static mpc_status solve_impl(mpc_plan_s* p, const mpc_problem_batch* b, hipStream_t s) {
  const SolverConsts sc{p->desc.rho, p->desc.sigma, p->desc.alpha, p->desc.rho_eq_scale,
                        p->desc.rho_min};
  const mpc_problem_batch sb = solver_batch(p, b);
  if (p->scaled) {
    PhaseTimer t(p, 0, s);
    HIP_TRY(launch_ruiz<T>(p->d_desc, p->n, make_inputs<T>(b), p->desc.scaling_iters,
                           scaled_out<T>(p), p->d_scale, b->warm_start, make_state<T>(p), s));
  }
  if (p->adaptive) HIP_TRY(launch_rho_init(p->d_rho, p->d_rho_hist, p->n, p->n_seg, p->desc.rho, s));
  const int K = p->desc.admm_iters;
  const int seg = p->adaptive ? p->desc.rho_interval : K;
  int warm = b->warm_start;
  // without scaling the last segment's groups check their own residuals (the
  // iterate is already the caller's); with it, after the unscaling below
  const bool group_res = !p->scaled;
  for (int done = 0, seg_i = 0; done < K; ++seg_i) {
    const int k = std::min(seg, K - done);
    mpc_status r = run_groups<T>(p, &sb, s, warm, k, group_res && done + k == K);
    if (r != MPC_OK) return r;
    done += k;
    warm = 1;
    if (p->adaptive && done < K) {
      PhaseTimer t(p, 2, s);
      HIP_TRY(launch_residual<T>(p->d_desc, nullptr, p->n, make_inputs<T>(&sb), sc,
                                 make_state<T>(p), p->lds_res, s));
      HIP_TRY(launch_rho_update<T>(p->d_desc, p->n, make_inputs<T>(&sb), make_state<T>(p),
                                   p->d_res, p->d_rho, p->desc.rho_tolerance, p->d_rho_hist,
                                   p->n_seg, seg_i + 1, s));
    }
  }
  if (p->scaled) {
    PhaseTimer t(p, 2, s);
    HIP_TRY(launch_unscale<T>(p->d_desc, p->n, p->d_scale, make_state<T>(p), s));
    HIP_TRY(launch_residual<T>(p->d_desc, nullptr, p->n, make_inputs<T>(b), sc, make_state<T>(p),
                               p->lds_res, s));
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_solve(mpc_plan_t p, const mpc_problem_batch* b, void* stream) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  mpc_status cs = check_batch(p, b);
  if (cs != MPC_OK) return cs;
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  p->last_stream = s;
  mpc_status r = p->fp64 ? solve_impl<double>(p, b, s) : solve_impl<float>(p, b, s);
  if (r == MPC_OK) p->solved = true;
  if (r == MPC_OK && p->kkt) p->kkt_state = true;
  return r;
}

extern "C" mpc_status mpc_get_solution(mpc_plan_t p, const mpc_solution* o, void* stream) {
  if (!p || !o) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solve has been issued on this plan");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  const size_t e = p->esz;
  if (o->x) HIP_TRY(hipMemcpyAsync(o->x, p->d_x, e * p->nX, hipMemcpyDeviceToDevice, s));
  if (o->u) HIP_TRY(hipMemcpyAsync(o->u, p->d_u, e * p->nU, hipMemcpyDeviceToDevice, s));
  if (o->z) HIP_TRY(hipMemcpyAsync(o->z, p->d_z, e * p->nZ, hipMemcpyDeviceToDevice, s));
  if (o->y) HIP_TRY(hipMemcpyAsync(o->y, p->d_y, e * p->nZ, hipMemcpyDeviceToDevice, s));
  if (o->objective) HIP_TRY(hipMemcpyAsync(o->objective, p->d_obj, e * p->n, hipMemcpyDeviceToDevice, s));
  if (o->residuals) HIP_TRY(hipMemcpyAsync(o->residuals, p->d_res, sizeof(double) * 4 * p->n, hipMemcpyDeviceToDevice, s));
  if (o->status) HIP_TRY(hipMemcpyAsync(o->status, p->d_status, sizeof(int32_t) * p->n, hipMemcpyDeviceToDevice, s));
  if (p->limits && o->zx) HIP_TRY(hipMemcpyAsync(o->zx, p->d_zx, e * p->nZX, hipMemcpyDeviceToDevice, s));
  if (p->limits && o->yx) HIP_TRY(hipMemcpyAsync(o->yx, p->d_yx, e * p->nZX, hipMemcpyDeviceToDevice, s));
  if (p->kkt && o->zd) HIP_TRY(hipMemcpyAsync(o->zd, p->d_zd, e * p->nC, hipMemcpyDeviceToDevice, s));
  if (p->kkt && o->yd) HIP_TRY(hipMemcpyAsync(o->yd, p->d_yd, e * p->nC, hipMemcpyDeviceToDevice, s));
  if (p->contacts && p->nZC > 0 && o->zc)
    HIP_TRY(hipMemcpyAsync(o->zc, p->d_zc, e * p->nZC, hipMemcpyDeviceToDevice, s));
  if (p->contacts && p->nZC > 0 && o->yc)
    HIP_TRY(hipMemcpyAsync(o->yc, p->d_yc, e * p->nZC, hipMemcpyDeviceToDevice, s));
  if (o->u0) {
    // u0 of agent a is the first nu entries of its u block: a strided copy
    // when every block has one size, else one gather kernel.
    if (p->uniform_u) {
      const size_t nu = p->hdesc[0].nu, N = p->hdesc[0].N;
      HIP_TRY(hipMemcpy2DAsync(o->u0, nu * e, p->d_u, N * nu * e, nu * e, p->n, hipMemcpyDeviceToDevice, s));
    } else if (p->fp64) {
      hipLaunchKernelGGL(k_gather_u0_packed<double>, dim3(p->n), dim3(64), 0, s, p->d_desc, p->d_u0off,
                         p->n, (const double*)p->d_u, (double*)o->u0);
      HIP_TRY(hipGetLastError());
    } else {
      hipLaunchKernelGGL(k_gather_u0_packed<float>, dim3(p->n), dim3(64), 0, s, p->d_desc, p->d_u0off,
                         p->n, (const float*)p->d_u, (float*)o->u0);
      HIP_TRY(hipGetLastError());
    }
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_set_warm_state(mpc_plan_t p, const void* u, const void* z, const void* y,
                                         void* stream) {
  if (!p || !u || !z || !y) return fail(MPC_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(p->d_u, u, p->esz * p->nU, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_z, z, p->esz * p->nZ, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_y, y, p->esz * p->nZ, hipMemcpyDeviceToDevice, s));
  p->solved = true;
  return MPC_OK;
}

extern "C" mpc_status mpc_set_warm_limits(mpc_plan_t p, const void* zx, const void* yx,
                                          void* stream) {
  if (!p || !zx || !yx) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->limits) return fail(MPC_ERR_INVALID_ARG, "this plan has no joint limits");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(p->d_zx, zx, p->esz * p->nZX, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_yx, yx, p->esz * p->nZX, hipMemcpyDeviceToDevice, s));
  return MPC_OK;
}

extern "C" mpc_status mpc_set_warm_kkt(mpc_plan_t p, const void* x, const void* zd, const void* yd,
                                        void* stream) {
  if (!p || !x || !zd || !yd) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->kkt) return fail(MPC_ERR_INVALID_ARG, "this plan does not run the KKT inner solve");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(p->d_x, x, p->esz * p->nX, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_zd, zd, p->esz * p->nC, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_yd, yd, p->esz * p->nC, hipMemcpyDeviceToDevice, s));
  p->kkt_state = true;
  return MPC_OK;
}

extern "C" mpc_status mpc_set_warm_contacts(mpc_plan_t p, const void* zc, const void* yc,
                                            void* stream) {
  if (!p || !zc || !yc) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->contacts) return fail(MPC_ERR_INVALID_ARG, "this plan has no no-slip rows");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  if (p->nZC > 0) {
    HIP_TRY(hipMemcpyAsync(p->d_zc, zc, p->esz * p->nZC, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_yc, yc, p->esz * p->nZC, hipMemcpyDeviceToDevice, s));
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_advance_state(mpc_plan_t p, const mpc_problem_batch* b, const void* noise,
                                        void* x0_next, void* stream) {
  if (!p || !b || !x0_next) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!b->A || !b->B || !b->c || !b->x0) return fail(MPC_ERR_INVALID_ARG, "null input pointer in batch");
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solution to apply");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  if (p->fp64) {
    HIP_TRY(launch_advance<double>(p->d_desc, nullptr, p->n, make_inputs<double>(b), (const double*)p->d_u,
                                   (const double*)noise, (double*)x0_next, s));
  } else {
    HIP_TRY(launch_advance<float>(p->d_desc, nullptr, p->n, make_inputs<float>(b), (const float*)p->d_u,
                                  (const float*)noise, (float*)x0_next, s));
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_set_timing(mpc_plan_t p, int32_t enable) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  p->timing = enable != 0;
  for (int i = 0; i < kPhases; ++i) {
    p->ms[i] = 0;
    p->launches[i] = 0;
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_get_timing(mpc_plan_t p, double* ms, int64_t* launches) {
  if (!p || !ms || !launches) return fail(MPC_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipSetDevice(p->desc.device));
  for (auto& pe : p->pending) {
    HIP_TRY(hipEventSynchronize(pe.second.second));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
    p->ms[pe.first] += t;
    p->launches[pe.first] += 1;
    p->ev_pool.push_back(pe.second.first);
    p->ev_pool.push_back(pe.second.second);
  }
  p->pending.clear();
  for (int i = 0; i < kPhases; ++i) {
    ms[i] = p->ms[i];
    launches[i] = p->launches[i];
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_get_config(mpc_plan_t p, int32_t* kernel, int32_t* threads,
                                          int32_t* lds) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  const Group& g = p->groups[0];
  if (kernel) *kernel = p->kernel;
  if (threads) *threads = g.family == 2 ? g.fthreads : g.gthreads;
  if (lds) *lds = (int32_t)(g.family == 2 ? g.flds : std::max(g.lds_factor, g.lds_admm));
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_get_rho(mpc_plan_t p, double* rho, int32_t* n_segments,
                                       void* stream) {
  if (!p || (!rho && !n_segments)) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->adaptive) return fail(MPC_ERR_INVALID_ARG, "this plan keeps rho fixed");
  if (n_segments) *n_segments = p->n_seg;
  if (!rho) return MPC_OK;
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solve has been issued on this plan");
  HIP_TRY(hipSetDevice(p->desc.device));
  HIP_TRY(hipMemcpyAsync(rho, p->d_rho_hist, sizeof(double) * p->n * p->n_seg,
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_get_scaling(mpc_plan_t p, double* scale, void* stream) {
  if (!p || !scale) return fail(MPC_ERR_INVALID_ARG, "null argument");
  if (!p->scaled) return fail(MPC_ERR_INVALID_ARG, "this plan does not scale");
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solve has been issued on this plan");
  HIP_TRY(hipSetDevice(p->desc.device));
  HIP_TRY(hipMemcpyAsync(scale, p->d_scale, sizeof(double) * kScaleStride * p->n,
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_export_factor(mpc_plan_t p, int32_t agent, void* K, void* Acl,
                                             void* Hinv, void* sv, void* stream) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  if (agent < 0 || agent >= p->n) return fail(MPC_ERR_INVALID_ARG, "agent index out of range");
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solve has been issued on this plan");
  for (const Group& g : p->groups)
    for (int i = 0; i < g.count; ++i)
      if (p->hlist[g.list_off + i] == agent && g.family == 2)
        return fail(MPC_ERR_UNSUPPORTED_SHAPE,
                    "this agent's operators are kept in the register-resident layout");
  if (!p->solved) return fail(MPC_ERR_NOT_READY, "no solve has been issued on this plan");
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  const AgentDesc& d = p->hdesc[agent];
  const size_t e = p->esz;
  const char* base = (const char*)p->d_ws + (size_t)d.ows * e;
  const size_t nK = (size_t)d.N * d.nu * d.nx, nA = (size_t)d.N * d.nx * d.nx,
               nH = (size_t)d.N * d.nu * d.nu, nS = (size_t)d.N * d.nx;
  if (K) HIP_TRY(hipMemcpyAsync(K, base, nK * e, hipMemcpyDeviceToDevice, s));
  if (Acl) HIP_TRY(hipMemcpyAsync(Acl, base + nK * e, nA * e, hipMemcpyDeviceToDevice, s));
  if (Hinv) HIP_TRY(hipMemcpyAsync(Hinv, base + (nK + nA) * e, nH * e, hipMemcpyDeviceToDevice, s));
  if (sv) HIP_TRY(hipMemcpyAsync(sv, base + (nK + nA + nH) * e, nS * e, hipMemcpyDeviceToDevice, s));
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_get_groups(mpc_plan_t p, mpc_group_info* out, int32_t cap,
                                          int32_t* n_groups) {
  if (!p || !n_groups || (cap > 0 && !out)) return fail(MPC_ERR_INVALID_ARG, "null argument");
  *n_groups = (int32_t)p->groups.size();
  for (int i = 0; i < (int)p->groups.size() && i < cap; ++i) {
    const Group& g = p->groups[i];
    mpc_group_info& o = out[i];
    o.family = g.family;
    o.N = g.N;
    o.nx = g.nx;
    o.nu = g.nu;
    o.n_feet = g.n_feet;
    o.n_agents = g.count;
    o.threads = g.family == 2 ? g.fthreads : g.gthreads;
    o.lds_bytes = (int32_t)(g.family == 2 ? g.flds : std::max(g.lds_factor, g.lds_admm));
  }
  return MPC_OK;
}

// Times every candidate launch configuration of every group on the caller's
// stream (cold solves of that group only) and keeps the fastest.
extern "C" mpc_status mpc_plan_autotune(mpc_plan_t p, const mpc_problem_batch* b, int32_t reps,
                                        void* stream) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  if (reps < 1 || reps > 1000) return fail(MPC_ERR_INVALID_ARG, "reps must be in 1..1000");
  mpc_problem_batch cold = b ? *b : mpc_problem_batch{};
  cold.warm_start = 0;
  mpc_status cs = check_batch(p, &cold);
  if (cs != MPC_OK) return cs;
  HIP_TRY(hipSetDevice(p->desc.device));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const bool timing = p->timing;
  p->timing = false;
  mpc_status r = MPC_OK;
  if (p->scaled) {  // the groups' trial solves run on the equilibrated problem
    if (p->fp64)
      HIP_TRY(launch_ruiz<double>(p->d_desc, p->n, make_inputs<double>(&cold), p->desc.scaling_iters,
                                  scaled_out<double>(p), p->d_scale, 0, make_state<double>(p), s));
    else
      HIP_TRY(launch_ruiz<float>(p->d_desc, p->n, make_inputs<float>(&cold), p->desc.scaling_iters,
                                 scaled_out<float>(p), p->d_scale, 0, make_state<float>(p), s));
  }
  if (p->adaptive) HIP_TRY(launch_rho_init(p->d_rho, p->d_rho_hist, p->n, p->n_seg, p->desc.rho, s));
  for (Group& g : p->groups) {
    struct Cand { int family, threads; };
    std::vector<Cand> cands;
    if (g.fused_ok) cands.push_back({2, g.fthreads});
    // MPC_FP32_MFMA is defined on the register-resident kernels only
    if (p->desc.precision != MPC_FP32_MFMA)
      for (int t : {256, 128, 64}) cands.push_back({g.family == 4 ? 4 : 1, t});
    float best = INFINITY;
    Cand pick = {g.family, g.family == 2 ? g.fthreads : g.gthreads};
    for (const Cand& c : cands) {
      Group trial = g;
      trial.family = c.family;
      if (c.family != 2) trial.gthreads = c.threads;
      const mpc_problem_batch tb = solver_batch(p, &cold);
      r = p->fp64 ? run_group<double>(p, trial, &tb, s, 0, p->desc.admm_iters)
                  : run_group<float>(p, trial, &tb, s, 0, p->desc.admm_iters);
      if (r != MPC_OK) break;
      hipError_t he = hipEventRecord(e0, s);
      for (int i = 0; i < reps && he == hipSuccess && r == MPC_OK; ++i)
        r = p->fp64 ? run_group<double>(p, trial, &tb, s, 0, p->desc.admm_iters)
                    : run_group<float>(p, trial, &tb, s, 0, p->desc.admm_iters);
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) r = fail(MPC_ERR_HIP, std::string("autotune timing: ") + hipGetErrorString(he));
      if (r != MPC_OK) break;
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    if (r != MPC_OK) break;
    g.family = pick.family;
    if (pick.family != 2) g.gthreads = pick.threads;
    g.est = best;
  }
  if (r == MPC_OK) assign_queues(p->groups, 1 + (int)p->aux.size());
  p->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  p->kernel = 0;
  for (const Group& g : p->groups) p->kernel |= g.family;
  // the resident iterates are those of partial cold solves now, and a
  // captured step would launch the old configuration
  p->solved = false;
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  return r;
}

extern "C" mpc_status mpc_plan_capture(mpc_plan_t p, const mpc_problem_batch* b, const void* noise,
                                       void* x0_next) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  mpc_status cs = check_batch(p, b);
  if (cs != MPC_OK) return cs;
  HIP_TRY(hipSetDevice(p->desc.device));
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  p->capturing = true;
  const bool was_solved = p->solved;
  mpc_status r = p->fp64 ? solve_impl<double>(p, b, p->cap_stream) : solve_impl<float>(p, b, p->cap_stream);
  if (r == MPC_OK && x0_next) {
    if (p->fp64)
      r = [&]() -> mpc_status {
        HIP_TRY(launch_advance<double>(p->d_desc, nullptr, p->n, make_inputs<double>(b),
                                       (const double*)p->d_u, (const double*)noise,
                                       (double*)x0_next, p->cap_stream));
        return MPC_OK;
      }();
    else
      r = [&]() -> mpc_status {
        HIP_TRY(launch_advance<float>(p->d_desc, nullptr, p->n, make_inputs<float>(b),
                                      (const float*)p->d_u, (const float*)noise, (float*)x0_next,
                                      p->cap_stream));
        return MPC_OK;
      }();
  }
  p->capturing = false;
  p->solved = was_solved;
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(p->cap_stream, &g);
  if (r != MPC_OK) {
    if (g) hipGraphDestroy(g);
    return r;
  }
  if (ee != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(MPC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  }
  p->graph = g;
  HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
  return MPC_OK;
}

extern "C" mpc_status mpc_plan_replay(mpc_plan_t p, void* stream) {
  if (!p) return fail(MPC_ERR_INVALID_ARG, "null plan");
  if (!p->gexec) return fail(MPC_ERR_NOT_READY, "no captured step on this plan");
  HIP_TRY(hipSetDevice(p->desc.device));
  HIP_TRY(hipGraphLaunch(p->gexec, (hipStream_t)stream));
  p->solved = true;
  if (p->kkt) p->kkt_state = true;
  return MPC_OK;
}
