/*
 * mpc.h -- C ABI of the batched MPC QP solver for AMD Instinct MI355X (gfx950).
 *
 * One call solves, for every agent of a batch, the linearised whole-body MPC
 * quadratic program that real-time iteration reduces the paper's MPC problem
 * to (one QP per control step; Sec. II-A and Sec. III-B, Eq. (OCP) and
 * Eq. (mpc_formulation)), re-posed as a linear time-varying QP:
 *
 *   min  sum_{k=1..N} 1/2 (x_k - r_k)' Q (x_k - r_k)
 *      + sum_{k=0..N-1} 1/2 (u_k - ubar_k)' R (u_k - ubar_k)
 *   s.t. x_0 = xbar0,   x_{k+1} = A_k x_k + B_k u_k + c_k,
 *        l_k <= C_k u_k <= h_k,
 *
 * with u = [tau (n_tau); foot wrenches or forces], C_k = [I; friction
 * pyramid], torque box +-tau_max, stance feet f_z >= 0 and pyramid facets
 * <= 0, swing feet forced to a zero wrench (contact rows of
 * Eq. (mpc_formulation), with the cone replaced by a 4-sided pyramid).
 *
 * Method: OSQP's ADMM (adopted in Sec. III-B; KKT system Eq. (kkt_system))
 * with the dynamics rows kept exact.  The x-update's KKT system is then an
 * equality-constrained LQR: a Riccati factor computed once per solve plays
 * the role of Eq. (ldl), and a backward/forward sweep per iteration plays the
 * role of Eqs. (backsolve_1)-(backsolve_2); projection and dual update follow
 * (Alg. 1, QP-iteration loop).
 *
 * Conventions
 *   - All array arguments of mpc_problem_batch / mpc_solution are DEVICE
 *     pointers on the plan's device, caller-owned, row-major, agents
 *     concatenated in agent order (a uniform batch is the plain
 *     [n_agents][N][...] tensor).  Per-agent sizes:
 *        A [N][nx][nx]   B [N][nx][nu]   c [N][nx]    q_diag [nx]  r_diag [nu]
 *        x_ref [N+1][nx] (row 0 unused)  x0 [nx]     tau_max [n_tau]
 *        mu [1]          stance [N][n_feet] (uint8, nonzero = stance)
 *        u_ref [N][nu] (optional input reference, may be NULL = 0)
 *     Floating-point arrays have the plan's "io type": double for
 *     MPC_FP64, float for every other precision.
 *   - Solution arrays: u0 [nu], x [N+1][nx], u [N][nu], z [N][m], y [N][m]
 *     (m = nu + 4 n_feet), objective [1] in the io type; residuals [4]
 *     double (primal, dual, dynamics, complementarity infinity norms);
 *     status [1] int32 (see MPC_AGENT_*).
 *   - Calls are asynchronous and stream-ordered on the given stream
 *     (a hipStream_t passed as void*, NULL = the null stream).  Inputs must
 *     stay valid until the stream has reached the solve.
 *   - API errors are returned as mpc_status and never abort the process;
 *     mpc_last_error() gives a thread-local message.  Numerical failure is
 *     per agent in status[] and never affects other agents.
 *   - A plan is not thread-safe; use one plan per stream.
 */
#ifndef MPC_H
#define MPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPC_OK = 0,
  MPC_ERR_INVALID_ARG = 1,
  MPC_ERR_OUT_OF_MEMORY = 2,
  MPC_ERR_HIP = 3,
  MPC_ERR_UNSUPPORTED_SHAPE = 4,
  MPC_ERR_BUSY = 5,
  MPC_ERR_NOT_READY = 6
} mpc_status;

typedef enum {
  MPC_FP64 = 0,        /* everything in double                                    */
  MPC_FP32 = 1,        /* float io, operators and ADMM iterations; the Riccati    */
                       /* factor runs in double and is rounded to float once, and */
                       /* H_k^{-1} h accumulates in double                        */
  MPC_BF16_REFINE = 2, /* float io; Riccati block products with bf16 operands on   */
                       /* the matrix cores (fp32 accumulation), fp64 stage-Hessian */
                       /* inverse; iterations as MPC_FP32 but rolled out under the */
                       /* exact dynamics, with up to max_refine_sweeps KKT-residual */
                       /* refinement sweeps per x-update                            */
  MPC_FP16_REFINE = 3, /* as MPC_BF16_REFINE with fp16 operands                    */
  MPC_FP32_REFINE = 4, /* as MPC_BF16_REFINE with fp32 operands on the fp32 matrix */
                       /* cores (v_mfma_f32_16x16x4f32)                             */
  MPC_FP32_MFMA = 5    /* as MPC_FP32 on the register-resident kernels, the factor's */
                       /* block products with fp32 operands on the fp32 matrix     */
                       /* cores (fp32 accumulation), the stage-Hessian inverse and */
                       /* K = -H^{-1} G in fp64; no refinement.  Every agent needs  */
                       /* a register-resident instantiation (UNSUPPORTED_SHAPE     */
                       /* otherwise); not with kernel = 1, joint limits, no-slip    */
                       /* rows, the KKT inner solve or the parallel-in-time factor  */
} mpc_precision;

/* per-agent numerical status */
enum { MPC_AGENT_OK = 0, MPC_AGENT_CONVERGED = 1, MPC_AGENT_NOT_PD = 2, MPC_AGENT_NONFINITE = 3,
       MPC_AGENT_SUPERSEDED = 4 /* served loop: replaced by a newer request, not solved */ };

/* Shape of one agent's QP.  nu must equal n_tau + n_feet * foot_dim;
 * foot_dim is 6 (wrench f_x,f_y,f_z,m_x,m_y,m_z) or 3 (force f_x,f_y,f_z).
 * Limits: 1 <= N <= 64, 1 <= nx <= 64, 1 <= nu <= 32, n_feet <= 8, and the
 * generic iteration kernel's vectors, 8 (2(N+1)nx + 4N nu + 2N m + 3N nx + nx
 * + N nu + 256) bytes, must fit one workgroup's LDS (160 KB on MI355X: N <= 43
 * for nx = 48, nu = 30, m = 38); plan creation returns UNSUPPORTED_SHAPE
 * otherwise. */
typedef struct {
  int32_t N, nx, nu, n_tau, n_feet, foot_dim;
} mpc_shape;

typedef struct {
  int32_t n_agents;         /* > 0                                                   */
  const mpc_shape* shapes;  /* HOST array [n_agents]; copied at plan creation          */
  int32_t precision;        /* mpc_precision                                           */
  int32_t admm_iters;       /* fixed iteration count K (> 0)                           */
  double rho;               /* ADMM penalty of inequality rows        (default 0.1)    */
  double sigma;             /* proximal weight on x and u             (default 1e-6)   */
  double alpha;             /* over-relaxation in (0, 2)              (default 1.6)    */
  double rho_eq_scale;      /* equality rows get rho_eq_scale * rho   (default 1e3)    */
  double rho_min;           /* rows with both bounds infinite         (default 1e-6)   */
  int32_t max_refine_sweeps;/* refinement sweeps per x-update, mixed precisions only   */
  double refine_tol;        /* stop refining at |r|_inf <= refine_tol * |b|_inf        */
  int32_t device;           /* HIP device ordinal                                      */
  int32_t kernel;           /* 0 = auto, 1 = generic kernels only, 2 = register-      */
                            /* resident kernels only (UNSUPPORTED_SHAPE if an agent has */
                            /* no instantiation: FP32, nx/nu 48/30 or 36/24, N <= 20),  */
                            /* 3 = as 2, the iterations of each shape class in one      */
                            /* persistent launch over every horizon (agents taken       */
                            /* longest first from a work queue) instead of one launch   */
                            /* per horizon bucket                                       */
  int32_t scaling_iters;    /* Ruiz equilibration rounds before the factor, Alg. 1's    */
                            /* scaling step (0 = off, default; at most 100)             */
  int32_t rho_interval;     /* adaptive rho (OSQP's residual balancing): iterations    */
                            /* between estimates, each followed by a refactorisation    */
                            /* (0 = fixed rho, default)                                 */
  double rho_tolerance;     /* adopt an estimate that moves rho by more than this      */
                            /* factor either way (default 5, >= 1)                      */
  int32_t joint_limits;     /* 1: every solve carries joint limits x_lo <= x_k <= x_hi  */
                            /* (Eq. (mpc_formulation)); the agents then run the generic */
                            /* kernels, FP64 or FP32 only, without scaling (default 0)  */
  int32_t no_slip;          /* 1: every solve carries the no-slip rows J_f v_k = 0 of   */
                            /* the feet in stance (Eq. (mpc_formulation)) on x_1..x_N,  */
                            /* stance of stage min(k, N-1); FP64 or FP32 only, without  */
                            /* scaling or the persistent launch (kernel = 3); generic   */
                            /* kernels, or with kernel = 2 the register-resident one    */
                            /* (FP32, shapes 48/30 with 2 <= N <= 10 and 36/24 with     */
                            /* 2 <= N <= 11; its FP32 chains carry the equality rows'   */
                            /* large duals: error to 2.4e-5 measured) (default 0)       */
  int32_t inner_solve;      /* 0: exact dynamics, Riccati factor and sweeps (default);  */
                            /* 1: the paper's form, dynamics as equality rows with      */
                            /* penalty rho_eq_scale * rho and the quasi-definite KKT    */
                            /* matrix of Eq. (kkt_system) factored once by LDL^T        */
                            /* (Eq. (ldl)) and solved by substitution (Eqs.             */
                            /* (backsolve_1)-(backsolve_2)); FP64 or FP32, fixed rho,   */
                            /* no scaling, joint limits or no-slip rows                 */
  int32_t riccati_scan;     /* 1: the generic path's Riccati factor by a parallel-in-   */
                            /* time scan over the stages (the backward recursion as a  */
                            /* product of maps P -> J + A'P(I + CP)^{-1}A, C = B Rt^-1 */
                            /* B', composed in ceil(log2(N + 1)) doubling rounds, each */
                            /* round one launch over every agent and stage; then each  */
                            /* stage's operators from P_{k+1}, stage-parallel): for    */
                            /* long horizons served with few agents; FP64 arithmetic, */
                            /* FP64 or FP32 io, nx <= 48, generic kernels, not with    */
                            /* inner_solve (default 0)                                  */
} mpc_plan_desc;

/* Fill *desc with the defaults above for n_agents agents of the given shapes. */
void mpc_plan_desc_default(mpc_plan_desc* desc);

typedef struct mpc_plan_s* mpc_plan_t;

/* Set-up of Alg. 1 for a fixed batch of QPs of the form of Eq. (mpc_formulation)
 * (one per agent, Sec. III-B).
 * Validate the description, copy the shapes, and allocate device workspace:
 * factors, resident warm-start state (u, z, y), solution and status buffers.
 * Errors: INVALID_ARG (bad pointer, count or constant), UNSUPPORTED_SHAPE
 * (shape outside the limits), OUT_OF_MEMORY, HIP. */
mpc_status mpc_plan_create(const mpc_plan_desc* desc, mpc_plan_t* out);

/* Release every device buffer of the plan (waits for the device). */
mpc_status mpc_plan_destroy(mpc_plan_t plan);

typedef struct {
  const void *A, *B, *c, *q_diag, *r_diag, *x_ref, *x0, *tau_max, *mu;
  const uint8_t* stance;
  const void* u_ref;   /* may be NULL */
  int32_t warm_start;  /* 0: u = z = y = 0;  1: start from the plan's resident (u, z, y) */
  /* joint limits of Eq. (mpc_formulation): x_lo <= x_k <= x_hi at stages 1..N, [nx]
   * per agent (io type; +-infinity where a component has no limit); required by
   * plans with joint_limits = 1, NULL otherwise */
  const void *x_lo, *x_hi;
  /* no-slip rows of Eq. (mpc_formulation): per agent the foot velocity Jacobian
   * rows [n_feet * foot_dim][nx] over the whole state (row-major, io type; the
   * rows of foot f are rows f*foot_dim .. f*foot_dim + foot_dim - 1), the same
   * at every stage; required by plans with no_slip = 1, NULL otherwise */
  const void* J_foot;
} mpc_problem_batch;

/* Alg. 1 for every agent, from the KKT data (f_KKT) to the end of the QP
 * iterations: the optional Ruiz equilibration (f_Ruiz), the factor in the
 * role of Eq. (ldl) (once per solve, Sec. III-B, and again after every rho
 * update), each iteration the role of Eqs. (backsolve_1)-(backsolve_2) plus
 * OSQP's projection and dual update (the ADMM of Eq. (kkt_system)).  With
 * scaling the iterations run on the equilibrated problem and the returned
 * (and resident) iterate is mapped back to the caller's variables; u_ref must
 * then be NULL (INVALID_ARG otherwise).
 * Solve every agent: stage penalties and bounds, Riccati factor (once), then
 * admm_iters iterations of back-sweep, rollout, relaxation, projection and
 * dual update, then the FP64 KKT residual check.  The solution stays
 * resident in the plan (it is the next warm start).  warm_start = 1 before
 * any solve (or after mpc_plan_create) is INVALID_ARG. */
mpc_status mpc_solve(mpc_plan_t plan, const mpc_problem_batch* batch, void* stream);

typedef struct {
  void *u0, *x, *u, *z, *y, *objective; /* io type; any may be NULL (not copied) */
  double* residuals;                    /* [n][4], may be NULL                   */
  int32_t* status;                      /* [n],    may be NULL                   */
  void *zx, *yx;                        /* joint-limit rows' (z_x, y_x) [N][nx],  */
                                        /* io type (plans with joint limits);    */
                                        /* may be NULL                           */
  void *zc, *yc;                        /* no-slip rows' (z_c, y_c) [N][n_feet*   */
                                        /* foot_dim], io type (plans with no-slip */
                                        /* rows); may be NULL                    */
  void *zd, *yd;                        /* dynamics rows' (z, y) [N][nx], io type */
                                        /* (plans with inner_solve = 1); may be  */
                                        /* NULL                                  */
} mpc_solution;

/* The QP solution Alg. 1 returns after its fixed iteration count; u_0 is
 * the input of the first stage, the one real-time iteration applies (Sec.
 * II-A).
 * Copy the resident solution into caller device buffers (stream-ordered).
 * NOT_READY if no solve has been issued. */
mpc_status mpc_get_solution(mpc_plan_t plan, const mpc_solution* out, void* stream);

/* Warm start of the next QP from a previous iterate (real-time iteration
 * solves one QP per control step, Sec. II-A, seeded by the last solution).
 * Replace the resident warm-start state with caller device buffers u [N][nu],
 * z [N][m], y [N][m] (io type), e.g. to resume a controller. */
mpc_status mpc_set_warm_state(mpc_plan_t plan, const void* u, const void* z, const void* y,
                              void* stream);

/* The joint-limit rows' part of the warm start (plans with joint limits):
 * z_x, y_x [N][nx] per agent (io type, device), e.g. to resume a controller
 * together with mpc_set_warm_state. */
mpc_status mpc_set_warm_limits(mpc_plan_t plan, const void* zx, const void* yx, void* stream);

/* The warm start of the paper-form inner solve (plans with inner_solve = 1,
 * Eq. (kkt_system)): its iterate also holds the states, which are not re-rolled
 * from xbar0, and the dynamics rows' (z, y).  x [N+1][nx] (x_0 is replaced by
 * the next batch's xbar0), zd, yd [N][nx] per agent (io type, device), beside
 * mpc_set_warm_state's u, z, y.  INVALID_ARG for other plans. */
mpc_status mpc_set_warm_kkt(mpc_plan_t plan, const void* x, const void* zd, const void* yd,
                            void* stream);

/* The no-slip rows' part of the warm start (plans with no-slip rows, the
 * stance constraint of Eq. (mpc_formulation)): z_c, y_c [N][n_feet*foot_dim]
 * per agent (io type, device).  INVALID_ARG for a plan without the rows. */
mpc_status mpc_set_warm_contacts(mpc_plan_t plan, const void* zc, const void* yc, void* stream);

/* The system step x_{i+1} = f(x_i, u_i) of Eq. (OCP), linearised as the QP's
 * first stage, driving a closed loop of control steps.
 * Closed-loop plant step of every agent under its own first stage:
 * x0_next = A_0 x0 + B_0 u_0 + c_0 + noise, with u_0 the resident solution's
 * first input.  noise may be NULL.  x0_next may alias x0. */
mpc_status mpc_advance_state(mpc_plan_t plan, const mpc_problem_batch* batch, const void* noise,
                             void* x0_next, void* stream);

/* Timing of the phases Table II times separately (factor, QP iterations)
 * plus the residual check.
 * Per-kernel timing: when enabled, every launch of a solve is bracketed by
 * HIP events on the stream it runs on.  mpc_plan_get_timing waits for those
 * events and returns the accumulated milliseconds and launch counts of
 * {stage setup + factor, ADMM iterations, KKT residual} in ms[0..2] /
 * launches[0..2], summed over launch groups (groups on different streams may
 * overlap in time).  Enabling resets the counters.  Replays of a captured
 * step are not timed. */
mpc_status mpc_plan_set_timing(mpc_plan_t plan, int32_t enable);
mpc_status mpc_plan_get_timing(mpc_plan_t plan, double* ms, int64_t* launches);

/* Which kernel families the plan runs as a bit mask (1 generic, 2
 * register-resident, 4 mixed precision) and the launch shape of its largest
 * launch group. */
mpc_status mpc_plan_get_config(mpc_plan_t plan, int32_t* kernel, int32_t* threads_per_agent,
                               int32_t* lds_bytes);

/* Alg. 1's scaling step and OSQP's rho adaptation as the last solve applied
 * them.  mpc_plan_get_rho copies the rho every agent ran each segment with
 * (double [n][n_segments], device; n_segments = ceil(admm_iters /
 * rho_interval), written to *n_segments) and mpc_plan_get_scaling every
 * agent's scale record (double [n][128], device: D_x at [0, nx), D_u at
 * [64, 64 + nu), the cost factor at 96).  NOT_READY before a solve,
 * INVALID_ARG if the plan does not adapt rho / scale. */
mpc_status mpc_plan_get_rho(mpc_plan_t plan, double* rho, int32_t* n_segments, void* stream);
mpc_status mpc_plan_get_scaling(mpc_plan_t plan, double* scale, void* stream);

/* The factor of Eq. (ldl)'s role, in Riccati form (gains, closed-loop
 * operators, stage-Hessian inverses).
 * Copy agent `agent`'s Riccati factor of the last solve into caller device
 * buffers (io type): K [N][nu][nx], A_cl [N][nx][nx] (= A_k + B_k K_k),
 * Hinv [N][nu][nu] (= H_k^{-1}), s [N][nx] (= P_{k+1} c_k); any may be NULL.
 * Only plans running the generic kernels keep the factor in device memory
 * (UNSUPPORTED_SHAPE otherwise).  For tests and diagnostics. */
mpc_status mpc_plan_export_factor(mpc_plan_t plan, int32_t agent, void* K, void* A_cl, void* Hinv,
                                  void* s, void* stream);

/* Launch groups.  A plan splits its agents into groups: agents of one shape
 * class (nx, nu, n_tau, n_feet, foot_dim) and, for the register-resident
 * kernels, one horizon N.  Each group is one factor launch and one iteration
 * launch; groups are spread over up to four streams that fork from and join
 * back into the solve's stream. */
typedef struct {
  int32_t family;    /* 1 generic, 2 register-resident, 4 mixed precision     */
  int32_t N;         /* horizon (longest in the group for generic groups)      */
  int32_t nx, nu, n_feet;
  int32_t n_agents;
  int32_t threads;   /* workgroup size of the iteration kernel                 */
  int32_t lds_bytes; /* dynamic LDS of the group's largest launch              */
} mpc_group_info;

/* Number of groups in *n_groups and the first min(cap, n) of them in out. */
mpc_status mpc_plan_get_groups(mpc_plan_t plan, mpc_group_info* out, int32_t cap,
                               int32_t* n_groups);

/* Launch configuration search for the parallel solve of Sec. III-D (one
 * kernel launch serves every agent of a group).
 * Autotuner: for every group, time each candidate launch configuration (the
 * register-resident kernels where the group has them; the generic kernels
 * with 256, 128 and 64 threads per workgroup) over `reps` cold solves of
 * that group's agents on `stream`, and keep the fastest.  Synchronous.
 * The batch's warm_start is ignored.  Afterwards the resident state is
 * undefined (the next solve must be cold) and a captured step is dropped. */
mpc_status mpc_plan_autotune(mpc_plan_t plan, const mpc_problem_batch* batch, int32_t reps,
                             void* stream);

/* One control step of the parallel MPC of Alg. 1 (solve, then the plant
 * step) as one replayable launch sequence.
 * Capture one control step into a HIP graph held by the plan: mpc_solve on
 * `batch` (with its warm_start flag) and, if x0_next is not NULL,
 * mpc_advance_state with `noise` and x0_next.  The graph records the pointer
 * values of batch, noise and x0_next: every replay reads the memory they
 * point to at replay time.  Capture runs on a stream of the plan's own and
 * launches nothing.  A new capture replaces the previous one. */
mpc_status mpc_plan_capture(mpc_plan_t plan, const mpc_problem_batch* batch, const void* noise,
                            void* x0_next);

/* Launch the captured step on `stream` (stream-ordered).  NOT_READY if no
 * step has been captured. */
mpc_status mpc_plan_replay(mpc_plan_t plan, void* stream);

/* ---------------------------------------------------------------------------
 * Served request loop (continuous batching).  Controllers submit single-QP
 * requests as they arrive, each controller with its own shape.  The server
 * keeps every solved controller's iterate (x, u, z, y) resident on the device
 * as the warm start of its next request, launches pending requests in batches
 * whenever one of max_inflight batch slots is free (requests arriving while
 * others run join the next batch), and admits work by an HBM budget: one
 * device arena of hbm_budget_bytes holds resident states and the factor
 * workspace of in-flight requests; when it is full the least recently used
 * idle controllers lose their resident state (their next solve is cold) and
 * requests that still do not fit wait.  A controller's requests run in
 * arrival order, one at a time.  Each request is solved exactly as the same
 * agent in a plan of the same precision: its result does not depend on the
 * other requests of its batch.  With supersede = 1 (for controllers whose
 * newest state makes an older one moot, as in receding-horizon control under
 * overload), a request still waiting when a newer request of the same
 * controller arrives is dropped: *status_out (if given) receives
 * MPC_AGENT_SUPERSEDED once a later batch launches, u0_out is not written, the
 * ticket is never reported by mpc_server_poll, and stats.superseded counts it;
 * the newer request then runs warm-started from the last solved one.
 * A server runs its batches on four streams of its own (one per hardware
 * queue of the process), split among its batch slots.
 * ------------------------------------------------------------------------- */
typedef struct mpc_server_s* mpc_server_t;

typedef struct {
  mpc_plan_desc solver;      /* precision, admm_iters, constants, refinement, device;   */
                             /* n_agents, shapes and kernel are ignored; scaling_iters,  */
                             /* rho_interval, joint_limits and no_slip must be 0         */
  int64_t hbm_budget_bytes;  /* device memory of the server (default 1 GiB)             */
  int32_t max_batch;         /* requests per batch (default 4096)                       */
  int32_t max_inflight;      /* batches on the device at once, 1..8 (default 3)        */
  int32_t supersede;         /* 1: a controller's queued request that a newer one of it  */
                             /* follows before it launches completes unsolved (default 0)*/
} mpc_server_desc;

typedef struct {
  int64_t submitted, completed, batches, evictions;
  int64_t pending, inflight;             /* requests waiting / on the device now       */
  int64_t resident_controllers, resident_bytes;
  int64_t arena_bytes, arena_free_bytes;
  int64_t superseded;                    /* requests completed unsolved (supersede = 1) */
} mpc_server_stats;

void mpc_server_desc_default(mpc_server_desc* desc);

/* Every request is one QP of Eq. (mpc_formulation) for one controller's
 * control step (real-time iteration, Sec. II-A), solved as in mpc_solve.
 * Allocates the arena and the batch slots (each with its own stream).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP. */
mpc_status mpc_server_create(const mpc_server_desc* desc, mpc_server_t* out);

/* Waits for the device and releases everything. */
mpc_status mpc_server_destroy(mpc_server_t server);

/* Seconds on the server's steady clock (zero at creation); arrival and
 * completion times use it. */
double mpc_server_clock(mpc_server_t server);

/* One controller's QP of Eq. (mpc_formulation) for its current control step
 * (Sec. II-A), to be solved by Alg. 1's iterations like an agent of a plan.
 * Queue one request of controller controller_id (any int64 key).  problem
 * holds DEVICE pointers to this controller's data for ONE agent in the
 * layouts of mpc_problem_batch, in the io type of the server's precision;
 * u_ref must be NULL; they must stay valid until the request completes.
 * problem->warm_start = 1 starts from the controller's resident iterate when
 * it has one (cold otherwise).  On completion u_0 [nu] is written to u0_out
 * and, if status_out is not NULL, the agent status to *status_out (device
 * pointers).  A controller keeps the shape of its first request.  Launches
 * work if a batch slot is free.  Errors: INVALID_ARG, UNSUPPORTED_SHAPE,
 * OUT_OF_MEMORY (one request of this shape exceeds the budget), HIP. */
mpc_status mpc_server_submit(mpc_server_t server, int64_t controller_id, const mpc_shape* shape,
                             const mpc_problem_batch* problem, void* u0_out, int32_t* status_out,
                             double t_arrival, int64_t* ticket);

/* As mpc_server_submit (one QP of Eq. (mpc_formulation) per request), for
 * n requests at once (arrays of n; status_out and tickets may be NULL). */
mpc_status mpc_server_submit_many(mpc_server_t server, int32_t n, const int64_t* controller_ids,
                                  const mpc_shape* shapes, const mpc_problem_batch* problems,
                                  void* const* u0_out, int32_t* const* status_out,
                                  const double* t_arrival, int64_t* tickets);

/* Completion of the QP solves of Alg. 1 issued for queued requests.
 * Non-blocking: retire finished batches, launch pending work into free
 * slots, and report up to cap completed (solved) tickets with their
 * completion times (server clock, taken from the batch's completion event). */
mpc_status mpc_server_poll(mpc_server_t server, int64_t* done_tickets, double* done_time,
                           int32_t cap, int32_t* n_done);

/* Blocks until every submitted request has completed or been superseded
 * (completions stay reportable by mpc_server_poll; superseded statuses are
 * written).  OUT_OF_MEMORY if pending requests can never fit the budget. */
mpc_status mpc_server_drain(mpc_server_t server);

/* The warm start real-time iteration carries to a controller's next QP
 * (Sec. II-A).
 * Copy a controller's resident iterate (x [N+1][nx], u [N][nu], z, y [N][m],
 * io type) to caller device buffers; any may be NULL.  BUSY while it has a
 * request on the device, NOT_READY if it has no resident state. */
mpc_status mpc_server_get_state(mpc_server_t server, int64_t controller_id, void* x, void* u,
                                void* z, void* y, void* stream);

mpc_status mpc_server_get_stats(mpc_server_t server, mpc_server_stats* out);

/* ---------------------------------------------------------------------------
 * Solve without any device allocation.  For callers that cannot allocate
 * device memory: work recorded under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It is mpc_solve for a batch of agents of
 * ONE shape with a register-resident instantiation ((nx, nu) = (48, 30) or
 * (36, 24), N <= 20), MPC_FP32 only, and no plan: desc gives n_agents,
 * shapes (host array, every entry equal), admm_iters and the solver
 * constants (precision must be MPC_FP32; kernel, refinement fields ignored;
 * scaling_iters, rho_interval, joint_limits and no_slip must be 0).
 * The per-agent descriptors, the launch list and the Riccati operators live
 * in a device array of MPC_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends (about 500 humanoid agents
 * at N = 10); a batch that needs more is rejected with UNSUPPORTED_SHAPE and
 * a message naming the limit.  The iterate lives in the caller's buffers:
 * out->x, u, z, y, objective, residuals and status are required (device
 * pointers, layouts of mpc_solution) and receive the solution; with
 * batch->warm_start = 1 the solve starts from the u, z, y those buffers hold
 * (a previous solution of the same batch shape).  out->u0 may be NULL.
 * Nothing is allocated and nothing needs clearing between calls (every
 * scratch byte a solve reads is written by that solve first), but every call
 * on one device uses that device's one scratch array: calls that overlap on
 * a device (concurrent streams, threads) race and corrupt each other.
 * Stream-ordered on `stream`.  Errors: INVALID_ARG, UNSUPPORTED_SHAPE, HIP.
 * ------------------------------------------------------------------------- */
#define MPC_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
mpc_status mpc_solve_noalloc(const mpc_plan_desc* desc, const mpc_problem_batch* batch,
                             const mpc_solution* out, void* stream);

/* Thread-local description of the last error returned on this thread. */
const char* mpc_last_error(void);

/* Library version string. */
const char* mpc_version(void);

/* ---------------------------------------------------------------------------
 * The real-time iteration's front and back end (Alg. 1's f_KKT and f_RNEA) on
 * a kinematic tree: one degree of freedom per body, bodies in topological
 * order, the first six a chain of three prismatic joints along the world axes
 * and three revolute joints (the floating base, so every coordinate is
 * additive), the others revolute or prismatic joints hanging from earlier
 * bodies.  A joint's frame sits at its offset in the parent frame with the
 * parent's orientation; a revolute joint rotates the body about its axis by
 * q, a prismatic one moves it along the axis.  Feet carry world-frame wrenches
 * at a contact point (force, then moment for foot_dim = 6).  State x = (q, qd)
 * (nx = 2 n_bodies), input u = (joint torques, foot wrenches) -- the QP's
 * layouts.  Device arrays (FP64 for mpc_rnea, the io type of the precision
 * argument otherwise); model arrays on the host.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_bodies;           /* 7..24                                              */
  int32_t n_feet, foot_dim;   /* <= 8 feet, foot_dim 3 or 6                         */
  double gravity;             /* along -z of the world                              */
  const int32_t* parent;      /* [n] (-1 for body 0)                                */
  const int32_t* joint_type;  /* [n] 0 revolute, 1 prismatic                        */
  const double* axis;         /* [n][3] unit joint axes                             */
  const double* offset;       /* [n][3] joint frame origin in the parent frame      */
  const double* mass;         /* [n]                                                */
  const double* com;          /* [n][3] centre of mass, body frame                  */
  const double* inertia;      /* [n][3] principal inertia about the centre of mass  */
  const double* armature;     /* [n] the joint's reflected actuator inertia, added  */
                              /* to M's diagonal (NULL: none; 0 for the base)      */
  const int32_t* foot_body;   /* [n_feet]                                           */
  const double* foot_offset;  /* [n_feet][3] contact point, foot body frame         */
} mpc_model_desc;

typedef struct mpc_model_s* mpc_model_t;

/* Validate the tree and copy it to the device (one allocation, freed by
 * mpc_model_destroy, which waits for the device first).  INVALID_ARG for a
 * malformed tree (order, joint types, axes, a non-positive mass or inertia
 * from the sixth body on, a negative one before, feet on the base),
 * UNSUPPORTED_SHAPE for one outside the size limits. */
mpc_status mpc_model_create(const mpc_model_desc* desc, int32_t device, mpc_model_t* out);
mpc_status mpc_model_destroy(mpc_model_t model);

/* Eq. (rnea): tau = M(q) qdd + h(q, qd) - J(q)' F for count configurations
 * (q, qd, qdd, tau [count][n], F [count][n_feet*foot_dim] or NULL). */
mpc_status mpc_rnea(mpc_model_t model, int32_t count, const double* q, const double* qd,
                    const double* qdd, const double* F, double* tau, void* stream);

/* f_KKT of Alg. 1: the QP data of every stage about (x_k, u_k), k = 0..N-1,
 * of the semi-implicit Euler step of Eq. (mpc_formulation) (qd+ = qd + dt
 * qdd(q, qd, u), q+ = q + dt qd+, qdd from M qdd = S'tau + J'F - h):
 * A_k = df/dx and B_k = df/du exactly (the derivatives of inverse dynamics in
 * closed form, mapped through M^-1), c_k = f(x_k, u_k) - A_k x_k - B_k u_k.
 * x [n][N+1][nx] and u [n][N][nu] in mpc_get_solution's layouts (x_N unused),
 * so a solve's trajectory feeds the next linearisation; A [n][N][nx][nx],
 * B [n][N][nx][nu], c [n][N][nx] in mpc_problem_batch's layouts for agents of
 * one shape.  precision: MPC_FP64 (double io) or MPC_FP32 (float io; the
 * arithmetic stays double).  status [n] (cleared by the caller): an agent with
 * a non-finite x_k or u_k gets MPC_AGENT_NONFINITE, else one whose mass
 * matrix fails to factor MPC_AGENT_NOT_PD; its A, B, c are then left as they
 * were or partly written.  J_foot (NULL to skip) [n][n_feet*foot_dim][nx]:
 * the no-slip rows of Eq. (mpc_formulation) at x_0 in mpc_problem_batch's
 * J_foot layout -- zero on the positions; on the velocities, per foot, the
 * contact point's world linear velocity and (6D feet) the foot's angular
 * velocity per unit qd. */
mpc_status mpc_linearize(mpc_model_t model, int32_t n_agents, int32_t N, double dt, int32_t precision,
                         const void* x, const void* u, void* A, void* B, void* c, void* J_foot,
                         int32_t* status, void* stream);

/* f_RNEA and Eq. (mpc_torque): from the first stages of a QP solution (x
 * [count][N+1][nx], u [count][N][nu], mpc_get_solution's layouts),
 * qdd* = (qd*_1 - qd*_0) / dt, tau_rnea = RNEA(q*_0, qd*_0, qdd*, F*) with F*
 * the wrench part of u*_0, and the joint torques
 * tau = kp (q*_0 - q) + kd (qd*_0 - qd) + tau_rnea ([count][n_bodies - 6];
 * x_meas [count][nx] the measured state (q, qd)).  precision as mpc_linearize. */
mpc_status mpc_rti_torque(mpc_model_t model, int32_t count, int32_t N, double dt, double kp, double kd,
                          int32_t precision, const void* x, const void* u, const void* x_meas,
                          void* tau, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MPC_H */
