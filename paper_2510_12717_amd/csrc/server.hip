// Served request loop of the C ABI (include/mpc.h, mpc_server_*): continuous
// batching of single-controller QP solves with device-resident warm state and
// admission by an HBM budget.
//
// Every controller that has been solved keeps its iterate (x, u, z, y) in a
// slot of one device arena; its next request starts from it (the warm start
// of real-time iteration, Sec. III-B).  Pending requests are launched in
// batches as soon as one of max_inflight batch slots is free: a batch takes
// the oldest request of every ready controller (one per controller, so a
// controller's requests run in arrival order), each with a factor workspace
// slot from the same arena.  When the arena is full, the least recently used
// idle controllers lose their resident state (their next solve is cold);
// requests that still do not fit wait for a running batch to finish.
//
// A batch runs the same kernels as a plan: agent descriptors point into the
// caller's per-request problem data (offsets from the lowest address of each
// field) and into the arena, and agents are grouped by kernel family and
// shape.  A gather kernel copies u_0 (and the status) of each request to the
// caller's buffers; an event marks the batch done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/mpc.h"
#include "fused.h"
#include "host_api.h"
#include "mpc_internal.h"
#include "server_arena.h"

using namespace mpc;

namespace {

constexpr int64_t kUnit = 256;  // arena allocation granule (bytes)

template <typename T>
__global__ void __launch_bounds__(64)
k_gather_u0(const AgentDesc* __restrict__ desc, int n, const T* __restrict__ u,
            const int32_t* __restrict__ status, void* const* __restrict__ u0_out,
            int32_t* const* __restrict__ status_out) {
  const int a = blockIdx.x;
  if (a >= n) return;
  const AgentDesc d = desc[a];
  T* dst = reinterpret_cast<T*>(u0_out[a]);
  for (int j = threadIdx.x; j < d.nu; j += blockDim.x) dst[j] = u[d.ou + j];
  if (threadIdx.x == 0 && status_out[a]) *status_out[a] = status[a];
}

// Writes v to *p[i] for every i < n (statuses of superseded requests).
__global__ void __launch_bounds__(256) k_mark_status(int32_t* const* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *p[i] = v;
}


struct Request {
  int64_t ticket = 0, ctrl = 0;
  mpc_problem_batch prob{};
  void* u0_out = nullptr;
  int32_t* status_out = nullptr;
  double t_arrival = 0;
};

struct Ctrl {
  mpc_shape shape{};
  int64_t state_off = -1;  // arena units
  int64_t state_units = 0;
  bool has_state = false;  // resident iterate valid
  bool busy = false;       // a request of it is on the device
  bool ready = false;      // listed in the ready queue
  bool idle = false;       // in the idle list: holds a state slot, not busy
  int64_t prev = -1, next = -1;  // idle-list neighbours (less / more recently used)
  std::deque<Request> queue;     // pending requests, arrival order
};

// Streams of one server: a process has four hardware queues on this device, so
// more streams would only share queues, and a batch's launch could then wait
// in a queue behind another batch's long launch.  With S batch slots each slot
// owns 4 / S of them (S <= 4; slots beyond four share one stream each, in
// turn); a batch starts and ends on its slot's first stream and forks its
// launch groups over the slot's streams, longest first onto the least loaded.
constexpr int kServerStreams = 4;

struct Slot {
  hipStream_t stream = nullptr;  // the shared stream its batch starts and ends on (not owned)
  hipEvent_t done = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join[kServerStreams - 1] = {};
  bool busy = false;
  uint64_t seq = 0;  // launch order of its batch
  // device
  AgentDesc* d_desc = nullptr;
  int32_t* d_list = nullptr;
  void** d_u0 = nullptr;
  int32_t** d_st_out = nullptr;
  int32_t* d_status = nullptr;
  void* d_obj = nullptr;
  double* d_res = nullptr;
  // pinned host staging
  AgentDesc* h_desc = nullptr;
  int32_t* h_list = nullptr;
  void** h_u0 = nullptr;
  int32_t** h_st_out = nullptr;
  int32_t* h_status = nullptr;
  // statuses of superseded requests written with this slot's next batch
  int32_t** h_sup = nullptr;
  int32_t** d_sup = nullptr;
  // the batch
  std::vector<Request> reqs;
  std::vector<int64_t> ws_off, ws_units;
};

}  // namespace

struct mpc_server_s {
  mpc_server_desc desc{};
  size_t esz = 4;
  bool fp64 = false;
  bool mixed = false;
  bool f32_products = false;  // MPC_FP32_MFMA: the register-resident factor's products in FP32
  char* arena_base = nullptr;
  int64_t arena_bytes = 0;
  Arena arena;
  hipStream_t streams[kServerStreams] = {};
  std::vector<Slot> slots;
  std::unordered_map<int64_t, Ctrl> ctrls;
  int64_t n_pending = 0;                         // requests queued, not yet launched
  std::deque<int32_t*> sup_status;               // superseded requests' status_out, not yet written
  uint64_t launch_seq = 0;                       // batches launched
  std::deque<int64_t> ready;                     // controllers whose head request may run
  int64_t idle_head = -1, idle_tail = -1;        // idle list, least recently used first
  std::deque<std::pair<int64_t, double>> done;   // completed, not yet reported
  int64_t next_ticket = 1;
  hipEvent_t ev_ref = nullptr;
  std::chrono::steady_clock::time_point t0;
  double t_ref = 0;  // server clock at ev_ref
  int lds_max = 0;
  mpc_server_stats stats{};
};

static double server_now(const mpc_server_s* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static int ctrl_m(const mpc_shape& s) { return s.nu + 4 * s.n_feet; }

static int64_t state_elems(const mpc_shape& s) {
  const int m = ctrl_m(s);
  return (int64_t)(s.N + 1) * s.nx + (int64_t)s.N * s.nu + 2 * (int64_t)s.N * m;
}

// Kernel family of one request: 2 register-resident, 4 mixed precision, 1 generic.
static int family_of(const mpc_server_s* sv, const mpc_shape& s) {
  if (sv->mixed) return 4;
  if (!sv->fp64 && fused_supported(s.N, s.nx, s.nu, s.n_feet)) return 2;
  return 1;
}

static int64_t ws_bytes(const mpc_server_s* sv, const mpc_shape& s) {
  if (family_of(sv, s) == 2) return (int64_t)fused_agent_floats(s.N, s.nx, s.nu) * 4;
  return generic_ws_elems(s.N, s.nx, s.nu, ctrl_m(s)) * (int64_t)sv->esz;
}

static int64_t to_units(int64_t bytes) { return (bytes + kUnit - 1) / kUnit; }

static void free_slot_buffers(Slot& sl) {
  if (sl.done) hipEventDestroy(sl.done);
  for (int i = 0; i < kServerStreams - 1; ++i)
    if (sl.ev_join[i]) hipEventDestroy(sl.ev_join[i]);
  if (sl.ev_fork) hipEventDestroy(sl.ev_fork);
  hipFree(sl.d_desc);
  hipFree(sl.d_list);
  hipFree(sl.d_u0);
  hipFree(sl.d_st_out);
  hipFree(sl.d_status);
  hipFree(sl.d_obj);
  hipFree(sl.d_res);
  hipHostFree(sl.h_desc);
  hipHostFree(sl.h_list);
  hipHostFree(sl.h_u0);
  hipHostFree(sl.h_st_out);
  hipHostFree(sl.h_status);
  hipHostFree(sl.h_sup);
  hipFree(sl.d_sup);
}

static void free_server(mpc_server_s* s) {
  if (!s) return;
  for (auto& sl : s->slots) free_slot_buffers(sl);
  for (hipStream_t& st : s->streams)
    if (st) hipStreamDestroy(st);
  hipFree(s->arena_base);
  if (s->ev_ref) hipEventDestroy(s->ev_ref);
  delete s;
}

extern "C" void mpc_server_desc_default(mpc_server_desc* d) {
  if (!d) return;
  memset(d, 0, sizeof(*d));
  mpc_plan_desc_default(&d->solver);
  d->hbm_budget_bytes = (int64_t)1 << 30;
  d->max_batch = 4096;
  d->max_inflight = 3;
}

extern "C" mpc_status mpc_server_create(const mpc_server_desc* desc, mpc_server_t* out) {
  if (!desc || !out) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const mpc_plan_desc& sd = desc->solver;
  if (sd.precision < MPC_FP64 || sd.precision > MPC_FP32_MFMA)
    return api_fail(MPC_ERR_INVALID_ARG, "unknown precision");
  if (sd.admm_iters <= 0) return api_fail(MPC_ERR_INVALID_ARG, "admm_iters must be > 0");
  if (!(sd.rho > 0) || !(sd.sigma >= 0) || !(sd.alpha > 0 && sd.alpha < 2) ||
      !(sd.rho_eq_scale > 0) || !(sd.rho_min > 0))
    return api_fail(MPC_ERR_INVALID_ARG, "solver constants out of range");
  if (sd.max_refine_sweeps < 0 || sd.max_refine_sweeps > 16 || !(sd.refine_tol >= 0))
    return api_fail(MPC_ERR_INVALID_ARG, "refinement settings out of range");
  if (sd.scaling_iters != 0 || sd.rho_interval != 0 || sd.joint_limits != 0 || sd.no_slip != 0 ||
      sd.inner_solve != 0 || sd.riccati_scan != 0)
    return api_fail(MPC_ERR_INVALID_ARG,
                    "the served loop runs the serial Riccati solve without scaling, joint limits or no-slip rows and with a fixed rho");
  if (desc->max_batch < 1 || desc->max_batch > (1 << 20) || desc->max_inflight < 1 ||
      desc->max_inflight > 8)
    return api_fail(MPC_ERR_INVALID_ARG, "max_batch must be in 1..2^20 and max_inflight in 1..8");
  if (desc->supersede != 0 && desc->supersede != 1)
    return api_fail(MPC_ERR_INVALID_ARG, "supersede must be 0 or 1");
  if (desc->hbm_budget_bytes <= 0) return api_fail(MPC_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
  int ndev = 0;
  MPC_HIP_TRY(hipGetDeviceCount(&ndev));
  if (sd.device < 0 || sd.device >= ndev) return api_fail(MPC_ERR_INVALID_ARG, "device ordinal out of range");
  MPC_HIP_TRY(hipSetDevice(sd.device));

  auto* s = new mpc_server_s();
  s->desc = *desc;
  s->desc.solver.n_agents = 0;
  s->desc.solver.shapes = nullptr;
  s->fp64 = sd.precision == MPC_FP64;
  s->mixed = refine_precision(sd.precision);
  s->f32_products = sd.precision == MPC_FP32_MFMA;
  s->esz = s->fp64 ? 8 : 4;
  const int B = desc->max_batch;
  // per-slot buffers come out of the budget first
  const int64_t per_slot = (int64_t)B * (sizeof(AgentDesc) + sizeof(int32_t) + 3 * sizeof(void*) +
                                         sizeof(int32_t) + 8 + 4 * sizeof(double));
  s->arena_bytes = desc->hbm_budget_bytes - per_slot * desc->max_inflight;
  s->arena_bytes = s->arena_bytes / kUnit * kUnit;
  if (s->arena_bytes < kUnit) {
    delete s;
    return api_fail(MPC_ERR_INVALID_ARG, "hbm_budget_bytes too small for max_batch x max_inflight");
  }
  hipError_t e = hipMalloc((void**)&s->arena_base, (size_t)s->arena_bytes);
  s->arena.init(s->arena_bytes / kUnit);
  for (hipStream_t& st : s->streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  s->slots.resize(desc->max_inflight);
  for (auto& sl : s->slots) {
    sl.stream = s->streams[0];
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev_fork, hipEventDisableTiming);
    for (int i = 0; i < kServerStreams - 1 && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&sl.ev_join[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_desc, sizeof(AgentDesc) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_list, sizeof(int32_t) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_u0, sizeof(void*) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_st_out, sizeof(int32_t*) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_status, sizeof(int32_t) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_obj, 8 * (size_t)B);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_res, sizeof(double) * 4 * B);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_desc, sizeof(AgentDesc) * B, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_list, sizeof(int32_t) * B, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_u0, sizeof(void*) * B, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_st_out, sizeof(int32_t*) * B, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_status, sizeof(int32_t) * B, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_sup, sizeof(int32_t*) * B);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_sup, sizeof(int32_t*) * B, hipHostMallocDefault);
  }
  int lds_max = 0;
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, sd.device);
  s->lds_max = lds_max;
  if (e == hipSuccess && !s->fp64) e = fused_set_limits();
  if (e == hipSuccess) e = hipEventCreate(&s->ev_ref);
  if (e == hipSuccess) e = hipEventRecord(s->ev_ref, s->streams[0]);
  if (e == hipSuccess) e = hipEventSynchronize(s->ev_ref);
  if (e != hipSuccess) {
    const mpc_status st = api_fail(e == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,
                                   std::string("server setup: ") + hipGetErrorString(e));
    free_server(s);
    return st;
  }
  s->t0 = std::chrono::steady_clock::now();
  s->t_ref = 0.0;
  *out = s;
  return MPC_OK;
}

extern "C" mpc_status mpc_server_destroy(mpc_server_t s) {
  if (!s) return api_fail(MPC_ERR_INVALID_ARG, "null server");
  hipSetDevice(s->desc.solver.device);
  for (hipStream_t st : s->streams)
    if (st) hipStreamSynchronize(st);
  free_server(s);
  return MPC_OK;
}

extern "C" double mpc_server_clock(mpc_server_t s) { return s ? server_now(s) : 0.0; }

// The idle list (intrusive, O(1)): controllers join at the most recently used
// end when their batch retires; eviction takes the least recently used.
static void idle_push(mpc_server_s* s, int64_t id, Ctrl& c) {
  c.prev = s->idle_tail;
  c.next = -1;
  c.idle = true;
  if (s->idle_tail >= 0) s->ctrls[s->idle_tail].next = id;
  else s->idle_head = id;
  s->idle_tail = id;
}
static void idle_remove(mpc_server_s* s, Ctrl& c) {
  if (!c.idle) return;
  if (c.prev >= 0) s->ctrls[c.prev].next = c.next;
  else s->idle_head = c.next;
  if (c.next >= 0) s->ctrls[c.next].prev = c.prev;
  else s->idle_tail = c.prev;
  c.prev = c.next = -1;
  c.idle = false;
}

static void mark_ready(mpc_server_s* s, int64_t id, Ctrl& c) {
  if (!c.ready && !c.busy && !c.queue.empty()) {
    c.ready = true;
    s->ready.push_back(id);
  }
}

static mpc_status submit_one(mpc_server_s* s, int64_t ctrl, const mpc_shape* shape,
                             const mpc_problem_batch* prob, void* u0_out, int32_t* status_out,
                             double t_arrival, int64_t* ticket) {
  if (!shape || !prob || !u0_out) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  const mpc_shape& sh = *shape;
  auto it = s->ctrls.find(ctrl);
  const bool known = it != s->ctrls.end();
  if (known) {
    // its shape passed every check below on its first request
    if (memcmp(&it->second.shape, &sh, sizeof(sh)) != 0)
      return api_fail(MPC_ERR_INVALID_ARG, "a controller keeps its shape");
  } else {
    if (sh.N < 1 || sh.N > 64 || sh.nx < 1 || sh.nx > 64 || sh.nu < 1 || sh.nu > 32 ||
        sh.n_feet < 0 || sh.n_feet > 8 || sh.n_tau < 0 || (sh.foot_dim != 3 && sh.foot_dim != 6) ||
        sh.nu != sh.n_tau + sh.n_feet * sh.foot_dim)
      return api_fail(MPC_ERR_UNSUPPORTED_SHAPE, "unsupported controller shape");
    if (s->mixed && !mixed_supported(sh.nx, sh.nu))
      return api_fail(MPC_ERR_UNSUPPORTED_SHAPE,
                      "mixed precision is built for (nx, nu) = (48, 30) and (36, 24) only");
    if (s->f32_products && !fused_supported(sh.N, sh.nx, sh.nu, sh.n_feet))
      return api_fail(MPC_ERR_UNSUPPORTED_SHAPE,
                      "MPC_FP32_MFMA needs a register-resident instantiation of the shape");
  }
  if (!prob->A || !prob->B || !prob->c || !prob->q_diag || !prob->r_diag || !prob->x_ref ||
      !prob->x0 || !prob->mu || (sh.n_tau > 0 && !prob->tau_max) || (sh.n_feet > 0 && !prob->stance))
    return api_fail(MPC_ERR_INVALID_ARG, "null input pointer in request");
  if (prob->u_ref) return api_fail(MPC_ERR_INVALID_ARG, "requests take no input reference (u_ref must be NULL)");
  if (prob->x_lo || prob->x_hi || prob->J_foot)
    return api_fail(MPC_ERR_INVALID_ARG,
                    "the served loop runs without joint limits or no-slip rows (x_lo, x_hi, J_foot must be NULL)");
  if (!known) {
    const int m = ctrl_m(sh);
    if ((int64_t)generic_admm_lds(sh.N, sh.nx, sh.nu, m, s->esz) > s->lds_max ||
        (int64_t)generic_factor_lds(sh.nx, sh.nu, s->esz) > s->lds_max)
      return api_fail(MPC_ERR_UNSUPPORTED_SHAPE, "controller shape needs more LDS than the device offers");
    // the generic kernels' LDS limits grow to what this shape needs
    MPC_HIP_TRY(generic_set_lds_limits(generic_factor_lds(sh.nx, sh.nu, s->esz),
                                       generic_admm_lds(sh.N, sh.nx, sh.nu, m, s->esz),
                                       generic_residual_lds(sh.N, sh.nx, sh.nu, s->esz)));
    const int64_t need = to_units(state_elems(sh) * (int64_t)s->esz) + to_units(ws_bytes(s, sh));
    if (need > s->arena_bytes / kUnit)
      return api_fail(MPC_ERR_OUT_OF_MEMORY, "one request of this shape exceeds the HBM budget");
    it = s->ctrls.emplace(ctrl, Ctrl{}).first;
    it->second.shape = sh;
  }
  Ctrl& c = it->second;
  if (s->desc.supersede && !c.queue.empty()) {
    // the waiting requests of this controller are moot: drop them
    for (const Request& old : c.queue)
      if (old.status_out) s->sup_status.push_back(old.status_out);
    s->n_pending -= (int64_t)c.queue.size();
    s->stats.superseded += (int64_t)c.queue.size();
    c.queue.clear();
  }
  c.queue.emplace_back();
  Request& r = c.queue.back();
  r.ticket = s->next_ticket++;
  r.ctrl = ctrl;
  r.prob = *prob;
  r.u0_out = u0_out;
  r.status_out = status_out;
  r.t_arrival = t_arrival;
  s->n_pending++;
  mark_ready(s, ctrl, c);
  if (ticket) *ticket = r.ticket;
  s->stats.submitted++;
  return MPC_OK;
}

// Evicts least recently used idle controllers until `units` can be allocated
// (high: a workspace slot, from the top of the arena).
static int64_t alloc_evicting(mpc_server_s* s, int64_t units, bool high = false) {
  auto take = [&]() { return high ? s->arena.alloc_high(units) : s->arena.alloc(units); };
  int64_t off = take();
  while (off < 0 && s->idle_head >= 0) {
    Ctrl& c = s->ctrls[s->idle_head];
    idle_remove(s, c);
    s->arena.release(c.state_off, c.state_units);
    c.state_off = -1;
    c.has_state = false;
    s->stats.evictions++;
    off = take();
  }
  return off;
}

template <typename T>
static Inputs<T> batch_inputs(const std::vector<Request>& reqs, std::vector<AgentDesc>& desc,
                              bool& misaligned) {
  // base of each field: the lowest address among the batch's requests
  auto base_of = [&](auto get) {
    uintptr_t b = UINTPTR_MAX;
    for (const auto& r : reqs) {
      const uintptr_t p = (uintptr_t)get(r.prob);
      if (p && p < b) b = p;
    }
    return b == UINTPTR_MAX ? (uintptr_t)0 : b;
  };
  auto off = [&](const void* p, uintptr_t base, size_t es) -> int64_t {
    if (!p) return 0;
    const uintptr_t d = (uintptr_t)p - base;
    if (d % es) misaligned = true;
    return (int64_t)(d / es);
  };
  Inputs<T> in{};
  const uintptr_t bA = base_of([](const mpc_problem_batch& b) { return b.A; });
  const uintptr_t bB = base_of([](const mpc_problem_batch& b) { return b.B; });
  const uintptr_t bc = base_of([](const mpc_problem_batch& b) { return b.c; });
  const uintptr_t bq = base_of([](const mpc_problem_batch& b) { return b.q_diag; });
  const uintptr_t br = base_of([](const mpc_problem_batch& b) { return b.r_diag; });
  const uintptr_t bxr = base_of([](const mpc_problem_batch& b) { return b.x_ref; });
  const uintptr_t bx0 = base_of([](const mpc_problem_batch& b) { return b.x0; });
  const uintptr_t bt = base_of([](const mpc_problem_batch& b) { return b.tau_max; });
  const uintptr_t bmu = base_of([](const mpc_problem_batch& b) { return b.mu; });
  const uintptr_t bst = base_of([](const mpc_problem_batch& b) { return (const void*)b.stance; });
  in.A = (const T*)bA;
  in.B = (const T*)bB;
  in.c = (const T*)bc;
  in.q = (const T*)bq;
  in.r = (const T*)br;
  in.xr = (const T*)bxr;
  in.x0 = (const T*)bx0;
  in.tau = (const T*)bt;
  in.mu = (const T*)bmu;
  in.st = (const uint8_t*)bst;
  in.uref = nullptr;
  for (size_t i = 0; i < reqs.size(); ++i) {
    const mpc_problem_batch& p = reqs[i].prob;
    AgentDesc& d = desc[i];
    d.oA = off(p.A, bA, sizeof(T));
    d.oB = off(p.B, bB, sizeof(T));
    d.oc = off(p.c, bc, sizeof(T));
    d.oq = off(p.q_diag, bq, sizeof(T));
    d.orr = off(p.r_diag, br, sizeof(T));
    d.oxr = off(p.x_ref, bxr, sizeof(T));
    d.ox0 = off(p.x0, bx0, sizeof(T));
    d.otau = off(p.tau_max, bt, sizeof(T));
    d.omu = off(p.mu, bmu, sizeof(T));
    d.ost = off(p.stance, bst, 1);
    d.our = 0;
  }
  return in;
}

// Up to max_batch pending superseded statuses, written on the slot's stream
// (the slot is idle: its staging buffer is free).
static mpc_status flush_superseded(mpc_server_s* s, Slot& sl) {
  const int n = (int)std::min<size_t>(s->sup_status.size(), (size_t)s->desc.max_batch);
  if (n == 0) return MPC_OK;
  for (int i = 0; i < n; ++i) {
    sl.h_sup[i] = s->sup_status.front();
    s->sup_status.pop_front();
  }
  MPC_HIP_TRY(hipMemcpyAsync(sl.d_sup, sl.h_sup, sizeof(int32_t*) * n, hipMemcpyHostToDevice, sl.stream));
  hipLaunchKernelGGL(k_mark_status, dim3((n + 255) / 256), dim3(256), 0, sl.stream, sl.d_sup, n,
                     (int32_t)MPC_AGENT_SUPERSEDED);
  MPC_HIP_TRY(hipGetLastError());
  return MPC_OK;
}

template <typename T>
static mpc_status launch_batch(mpc_server_s* s, Slot& sl) {
  const int n = (int)sl.reqs.size();
  std::vector<AgentDesc> desc(n);
  bool misaligned = false;
  Inputs<T> in = batch_inputs<T>(sl.reqs, desc, misaligned);
  if (misaligned) return api_fail(MPC_ERR_INVALID_ARG, "request arrays are not element-aligned");
  const SolverConsts sc{s->desc.solver.rho, s->desc.solver.sigma, s->desc.solver.alpha,
                        s->desc.solver.rho_eq_scale, s->desc.solver.rho_min};
  // groups: (family, nx, nu, n_tau, n_feet, foot_dim, horizon bucket for register-resident)
  std::map<std::tuple<int, int, int, int, int, int, int>, std::vector<int32_t>> groups;
  for (int i = 0; i < n; ++i) {
    const Request& r = sl.reqs[i];
    Ctrl& c = s->ctrls[r.ctrl];
    const mpc_shape& sh = c.shape;
    AgentDesc& d = desc[i];
    d.N = sh.N;
    d.nx = sh.nx;
    d.nu = sh.nu;
    d.n_tau = sh.n_tau;
    d.n_feet = sh.n_feet;
    d.foot_dim = sh.foot_dim;
    d.m = ctrl_m(sh);
    const int64_t base = c.state_off * kUnit / (int64_t)s->esz;
    d.ox = base;
    d.ou = d.ox + (int64_t)(sh.N + 1) * sh.nx;
    d.oz = d.ou + (int64_t)sh.N * sh.nu;
    d.oy = d.oz + (int64_t)sh.N * d.m;
    d.flags = (r.prob.warm_start && c.has_state) ? AGENT_FLAG_WARM : 0;
    const int fam = family_of(s, sh);
    const int64_t wb = sl.ws_off[i] * kUnit;
    d.ows = wb / (int64_t)s->esz;
    d.ofw = fam == 2 ? wb / 4 : -1;
    groups[std::make_tuple(fam, sh.nx, sh.nu, sh.n_tau, sh.n_feet, sh.foot_dim,
                           fam == 2 ? fused_bucket(sh.N) : 0)]
        .push_back(i);
    sl.h_u0[i] = r.u0_out;
    sl.h_st_out[i] = r.status_out;
  }
  memcpy(sl.h_desc, desc.data(), sizeof(AgentDesc) * n);
  int pos = 0;
  struct G { int fam, N, nx, nu, n_feet, off, count; size_t lds_f, lds_a; };
  std::vector<G> gl;
  for (auto& kv : groups) {
    std::vector<int32_t>& v = kv.second;
    // longest horizon first so the tail of a launch is short
    std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) { return desc[x].N > desc[y].N; });
    G g{std::get<0>(kv.first), 0, std::get<1>(kv.first), std::get<2>(kv.first),
        std::get<4>(kv.first), pos, (int)v.size(), 0, 0};
    for (int32_t i : v) {
      sl.h_list[pos++] = i;
      g.N = std::max(g.N, desc[i].N);
    }
    g.lds_f = generic_factor_lds(g.nx, g.nu, s->esz);
    g.lds_a = generic_admm_lds(g.N, g.nx, g.nu, g.nu + 4 * g.n_feet, s->esz);
    gl.push_back(g);
  }
  const int n_slots = (int)s->slots.size();
  const int per_slot = std::max(1, kServerStreams / n_slots);
  const int base = (int)((&sl - s->slots.data()) * per_slot % kServerStreams);
  sl.stream = s->streams[base];
  hipStream_t st = sl.stream;
  {
    const mpc_status fr = flush_superseded(s, sl);
    if (fr != MPC_OK) return fr;
  }
  MPC_HIP_TRY(hipMemcpyAsync(sl.d_desc, sl.h_desc, sizeof(AgentDesc) * n, hipMemcpyHostToDevice, st));
  MPC_HIP_TRY(hipMemcpyAsync(sl.d_list, sl.h_list, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  MPC_HIP_TRY(hipMemcpyAsync(sl.d_u0, sl.h_u0, sizeof(void*) * n, hipMemcpyHostToDevice, st));
  MPC_HIP_TRY(hipMemcpyAsync(sl.d_st_out, sl.h_st_out, sizeof(int32_t*) * n, hipMemcpyHostToDevice, st));
  State<T> state{(T*)s->arena_base, (T*)s->arena_base, (T*)s->arena_base, (T*)s->arena_base,
                 (T*)sl.d_obj, sl.d_res, sl.d_status};
  const int iters = s->desc.solver.admm_iters;
  // groups spread over the slot's streams, forked from and joined back into its
  // own; longest group first onto the stream with the least work so far
  auto cost = [](const G& g) { return (int64_t)g.count * g.N * (g.nx + g.nu); };
  std::stable_sort(gl.begin(), gl.end(), [&](const G& x, const G& y) { return cost(x) > cost(y); });
  const int ns = std::min<int>(per_slot, (int)gl.size());
  auto aux = [&](int i) { return s->streams[(base + 1 + i) % kServerStreams]; };
  std::vector<int64_t> load(ns, 0);
  if (ns > 1) {
    MPC_HIP_TRY(hipEventRecord(sl.ev_fork, sl.stream));
    for (int i = 0; i < ns - 1; ++i) MPC_HIP_TRY(hipStreamWaitEvent(aux(i), sl.ev_fork, 0));
  }
  for (size_t gi = 0; gi < gl.size(); ++gi) {
    const G& g = gl[gi];
    const int32_t* list = sl.d_list + g.off;
    const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[si] += cost(g);
    hipStream_t st = si == 0 ? sl.stream : aux(si - 1);
    if constexpr (std::is_same<T, float>::value) {
      if (g.fam == 2) {
        MPC_HIP_TRY(fused_solve_f32(sl.d_desc, list, g.count, g.N, g.nx, g.nu, g.n_feet, in, sc,
                                    iters, -1, state, (float*)s->arena_base, st, 3, nullptr,
                                    s->f32_products));
        continue;
      }
      if (g.fam == 4) {
        MPC_HIP_TRY(launch_mixed_factor(sl.d_desc, list, g.count, g.nx, g.nu,
                                        refine_product(s->desc.solver.precision), in, sc,
                                        (float*)s->arena_base, sl.d_status, st));
        MPC_HIP_TRY(launch_generic_admm<float>(sl.d_desc, list, g.count, in, sc, iters, -1,
                                               (const float*)s->arena_base, state, g.lds_a, 256,
                                               st, s->desc.solver.max_refine_sweeps,
                                               s->desc.solver.refine_tol));
        continue;
      }
    }
    if (!s->fp64 && mixed_supported(g.nx, g.nu))
      MPC_HIP_TRY(launch_mixed_factor(sl.d_desc, list, g.count, g.nx, g.nu, 0,
                                      *reinterpret_cast<const Inputs<float>*>(&in), sc,
                                      (float*)s->arena_base, sl.d_status, st));
    else
      MPC_HIP_TRY(launch_generic_factor<T>(sl.d_desc, list, g.count, in, sc, (T*)s->arena_base,
                                           sl.d_status, g.lds_f, 256, st));
    MPC_HIP_TRY(launch_generic_admm<T>(sl.d_desc, list, g.count, in, sc, iters, -1,
                                       (const T*)s->arena_base, state, g.lds_a, 256, st));
  }
  for (int i = 0; i < ns - 1; ++i) {
    MPC_HIP_TRY(hipEventRecord(sl.ev_join[i], aux(i)));
    MPC_HIP_TRY(hipStreamWaitEvent(sl.stream, sl.ev_join[i], 0));
  }
  st = sl.stream;
  int maxN = 1, maxnx = 1, maxnu = 1;
  for (const G& g : gl) {
    maxN = std::max(maxN, g.N);
    maxnx = std::max(maxnx, g.nx);
    maxnu = std::max(maxnu, g.nu);
  }
  MPC_HIP_TRY(launch_residual<T>(sl.d_desc, nullptr, n, in, sc, state,
                                 generic_residual_lds(maxN, maxnx, maxnu, s->esz), st));
  hipLaunchKernelGGL(k_gather_u0<T>, dim3(n), dim3(64), 0, st, sl.d_desc, n, (const T*)s->arena_base,
                     sl.d_status, sl.d_u0, sl.d_st_out);
  MPC_HIP_TRY(hipGetLastError());
  MPC_HIP_TRY(hipMemcpyAsync(sl.h_status, sl.d_status, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  MPC_HIP_TRY(hipEventRecord(sl.done, st));
  return MPC_OK;
}

// Forms and launches batches while a slot is free and requests are ready.
static mpc_status pump(mpc_server_s* s) {
  for (auto& sl : s->slots) {
    if (sl.busy) continue;
    if (s->ready.empty()) break;
    sl.reqs.clear();
    sl.ws_off.clear();
    sl.ws_units.clear();
    std::deque<int64_t> skipped;
    while (!s->ready.empty() && (int)sl.reqs.size() < s->desc.max_batch) {
      const int64_t id = s->ready.front();
      s->ready.pop_front();
      Ctrl& c = s->ctrls[id];
      c.ready = false;
      if (c.busy || c.queue.empty()) continue;
      // resident state slot (kept if it has one), then a workspace slot
      if (c.state_off < 0) {
        const int64_t su = to_units(state_elems(c.shape) * (int64_t)s->esz);
        const int64_t off = alloc_evicting(s, su);
        if (off < 0) {
          skipped.push_back(id);
          break;
        }
        c.state_off = off;
        c.state_units = su;
        c.has_state = false;
      } else {
        idle_remove(s, c);
      }
      const int64_t wu = to_units(ws_bytes(s, c.shape));
      const int64_t woff = alloc_evicting(s, wu, true);
      if (woff < 0) {
        // put the controller back (into the idle list at its most recently used
        // end: its request is waiting, so its state is evicted last)
        if (c.has_state) idle_push(s, id, c);
        else {
          s->arena.release(c.state_off, c.state_units);
          c.state_off = -1;
        }
        skipped.push_back(id);
        break;
      }
      c.busy = true;
      sl.reqs.push_back(c.queue.front());
      c.queue.pop_front();
      s->n_pending--;
      sl.ws_off.push_back(woff);
      sl.ws_units.push_back(wu);
    }
    for (auto it = skipped.rbegin(); it != skipped.rend(); ++it) {
      Ctrl& c = s->ctrls[*it];
      if (!c.ready) {
        c.ready = true;
        s->ready.push_front(*it);
      }
    }
    if (sl.reqs.empty()) break;
    const mpc_status r = s->fp64 ? launch_batch<double>(s, sl) : launch_batch<float>(s, sl);
    if (r != MPC_OK) return r;
    sl.busy = true;
    sl.seq = ++s->launch_seq;
    s->stats.batches++;
  }
  return MPC_OK;
}

// Retires finished batches; with wait, first waits for the oldest running one
// (only: the others keep running while the freed slot takes the next batch).
static mpc_status retire(mpc_server_s* s, bool wait) {
  if (wait) {
    Slot* oldest = nullptr;
    for (auto& sl : s->slots)
      if (sl.busy && (!oldest || sl.seq < oldest->seq)) oldest = &sl;
    if (oldest) MPC_HIP_TRY(hipEventSynchronize(oldest->done));
  }
  for (auto& sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    MPC_HIP_TRY(q);
    float ms = 0;
    MPC_HIP_TRY(hipEventElapsedTime(&ms, s->ev_ref, sl.done));
    const double t_done = s->t_ref + ms * 1e-3;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
      const Request& r = sl.reqs[i];
      Ctrl& c = s->ctrls[r.ctrl];
      c.busy = false;
      c.has_state = sl.h_status[i] == AGENT_OK;
      idle_push(s, r.ctrl, c);
      s->arena.release(sl.ws_off[i], sl.ws_units[i]);
      mark_ready(s, r.ctrl, c);
      s->done.push_back({r.ticket, t_done});
      s->stats.completed++;
    }
    sl.reqs.clear();
    sl.busy = false;
  }
  return MPC_OK;
}

extern "C" mpc_status mpc_server_submit(mpc_server_t s, int64_t controller_id, const mpc_shape* shape,
                                        const mpc_problem_batch* problem, void* u0_out,
                                        int32_t* status_out, double t_arrival, int64_t* ticket) {
  if (!s) return api_fail(MPC_ERR_INVALID_ARG, "null server");
  MPC_HIP_TRY(hipSetDevice(s->desc.solver.device));
  mpc_status r = submit_one(s, controller_id, shape, problem, u0_out, status_out, t_arrival, ticket);
  if (r != MPC_OK) return r;
  r = retire(s, false);
  if (r != MPC_OK) return r;
  return pump(s);
}

extern "C" mpc_status mpc_server_submit_many(mpc_server_t s, int32_t n, const int64_t* controller_ids,
                                             const mpc_shape* shapes,
                                             const mpc_problem_batch* problems, void* const* u0_out,
                                             int32_t* const* status_out, const double* t_arrival,
                                             int64_t* tickets) {
  if (!s) return api_fail(MPC_ERR_INVALID_ARG, "null server");
  if (n < 0 || (n > 0 && (!controller_ids || !shapes || !problems || !u0_out || !t_arrival)))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  MPC_HIP_TRY(hipSetDevice(s->desc.solver.device));
  for (int i = 0; i < n; ++i) {
    mpc_status r = submit_one(s, controller_ids[i], &shapes[i], &problems[i], u0_out[i],
                              status_out ? status_out[i] : nullptr, t_arrival[i],
                              tickets ? &tickets[i] : nullptr);
    if (r != MPC_OK) return r;
  }
  mpc_status r = retire(s, false);
  if (r != MPC_OK) return r;
  return pump(s);
}

extern "C" mpc_status mpc_server_poll(mpc_server_t s, int64_t* done_tickets, double* done_time,
                                      int32_t cap, int32_t* n_done) {
  if (!s || !n_done || (cap > 0 && !done_tickets)) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  MPC_HIP_TRY(hipSetDevice(s->desc.solver.device));
  mpc_status r = retire(s, false);
  if (r == MPC_OK) r = pump(s);
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    done_tickets[k] = s->done.front().first;
    if (done_time) done_time[k] = s->done.front().second;
    s->done.pop_front();
    ++k;
  }
  *n_done = k;
  return r;
}

extern "C" mpc_status mpc_server_drain(mpc_server_t s) {
  if (!s) return api_fail(MPC_ERR_INVALID_ARG, "null server");
  MPC_HIP_TRY(hipSetDevice(s->desc.solver.device));
  for (;;) {
    mpc_status r = pump(s);
    if (r != MPC_OK) return r;
    bool any = false;
    for (auto& sl : s->slots) any |= sl.busy;
    if (!any) {
      if (s->n_pending == 0) {
        // every slot is idle: write the superseded statuses still waiting
        s->slots[0].stream = s->streams[0];
        while (!s->sup_status.empty()) {
          r = flush_superseded(s, s->slots[0]);
          if (r != MPC_OK) return r;
          MPC_HIP_TRY(hipStreamSynchronize(s->streams[0]));
        }
        return MPC_OK;
      }
      return api_fail(MPC_ERR_OUT_OF_MEMORY, "pending requests do not fit the HBM budget");
    }
    r = retire(s, true);
    if (r != MPC_OK) return r;
  }
}

extern "C" mpc_status mpc_server_get_state(mpc_server_t s, int64_t controller_id, void* x, void* u,
                                           void* z, void* y, void* stream) {
  if (!s) return api_fail(MPC_ERR_INVALID_ARG, "null server");
  auto it = s->ctrls.find(controller_id);
  if (it == s->ctrls.end()) return api_fail(MPC_ERR_INVALID_ARG, "unknown controller");
  const Ctrl& c = it->second;
  if (c.busy) return api_fail(MPC_ERR_BUSY, "the controller has a request on the device");
  if (!c.has_state) return api_fail(MPC_ERR_NOT_READY, "the controller has no resident state");
  MPC_HIP_TRY(hipSetDevice(s->desc.solver.device));
  const mpc_shape& sh = c.shape;
  const size_t e = s->esz;
  const char* b = s->arena_base + c.state_off * kUnit;
  const size_t nxs = (size_t)(sh.N + 1) * sh.nx, nus = (size_t)sh.N * sh.nu,
               nzs = (size_t)sh.N * ctrl_m(sh);
  hipStream_t st = (hipStream_t)stream;
  if (x) MPC_HIP_TRY(hipMemcpyAsync(x, b, nxs * e, hipMemcpyDeviceToDevice, st));
  if (u) MPC_HIP_TRY(hipMemcpyAsync(u, b + nxs * e, nus * e, hipMemcpyDeviceToDevice, st));
  if (z) MPC_HIP_TRY(hipMemcpyAsync(z, b + (nxs + nus) * e, nzs * e, hipMemcpyDeviceToDevice, st));
  if (y) MPC_HIP_TRY(hipMemcpyAsync(y, b + (nxs + nus + nzs) * e, nzs * e, hipMemcpyDeviceToDevice, st));
  return MPC_OK;
}

extern "C" mpc_status mpc_server_get_stats(mpc_server_t s, mpc_server_stats* out) {
  if (!s || !out) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  *out = s->stats;
  out->pending = s->n_pending;
  int64_t inflight = 0;
  for (auto& sl : s->slots) inflight += (int64_t)sl.reqs.size();
  out->inflight = inflight;
  int64_t resident = 0, n_res = 0;
  for (auto& kv : s->ctrls)
    if (kv.second.state_off >= 0) {
      resident += kv.second.state_units * kUnit;
      ++n_res;
    }
  out->resident_bytes = resident;
  out->resident_controllers = n_res;
  out->arena_bytes = s->arena_bytes;
  out->arena_free_bytes = s->arena.free_units() * kUnit;
  return MPC_OK;
}
