/*
 * FP64 CPU oracle for the batched MPC QP solve -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this library.  The product path (the HIP library and
 * its binding) never calls it and shares no code with it.
 *
 * What it computes (one QP per agent, real-time iteration: Sec. II-A and
 * Sec. III-B of the paper), in the paper's notation re-posed as a linear
 * time-varying QP:
 *
 *   min  sum_{k=1..N} 1/2 (x_k - r_k)' Q (x_k - r_k)
 *      + sum_{k=0..N-1} 1/2 (u_k - ubar_k)' R (u_k - ubar_k)
 *   s.t. x_0 = xbar0,  x_{k+1} = A_k x_k + B_k u_k + c_k,
 *        l_k <= C_k u_k <= h_k                      (k = 0..N-1)
 *
 * C_k stacks an identity on u (torque box, contact wrench bounds) and a
 * four-sided friction pyramid per foot (linearised contact cone of
 * Eq. (mpc_formulation), Sec. III-A).
 *
 * It is solved with the ADMM iteration of OSQP that Sec. III-B adopts
 * (Eq. (kkt_system)), with the dynamics rows kept exact so that the KKT
 * system of each x-update is an equality-constrained LQR.  Its factor plays
 * the role of Eq. (ldl) (computed once per solve) and its two sweeps the role
 * of Eqs. (backsolve_1)-(backsolve_2) (repeated every iteration), as in
 * Alg. 1.  All arithmetic is IEEE double.
 */
#ifndef MPC_ORACLE_H
#define MPC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t N, nx, nu, n_tau, n_feet, foot_dim;
} orc_shape;

typedef struct {
  double rho;           /* ADMM penalty on inequality rows                    */
  double sigma;         /* proximal weight on the primal variables            */
  double alpha;         /* over-relaxation                                    */
  double rho_eq_scale;  /* penalty multiplier for equality rows (l == h)      */
  double rho_min;       /* penalty for rows with both bounds infinite         */
} orc_settings;

/* status codes per agent */
enum { ORC_OK = 0, ORC_CONVERGED = 1, ORC_NOT_PD = 2, ORC_NONFINITE = 3 };

/* m = nu + 4 * n_feet */
int32_t orc_rows(const orc_shape* s);

/* Dense constraint matrix C_k (m x nu, row-major) for friction coefficient mu. */
void orc_constraint_matrix(const orc_shape* s, double mu, double* C);

/* Bounds and per-row penalties of every stage: l, h, rho are [N][m]. */
void orc_stage_bounds(const orc_shape* s, const orc_settings* st, const double* tau_max,
                      const uint8_t* stance, double* l, double* h, double* rho);

/* Penalties rho_x [nx] of the state rows (joint limits x_lo <= x_k <= x_hi). */
void orc_state_penalties(const orc_shape* s, const orc_settings* st, const double* x_lo,
                         const double* x_hi, double* rho_x);

/* no-slip rows per stage: n_feet * foot_dim */
int32_t orc_contact_rows(const orc_shape* s);

/* Bounds and penalties [N][nc] of the no-slip rows of x_1..x_N (stance of
 * stage min(k, N-1): equality rows; swing: free rows). */
void orc_contact_bounds(const orc_shape* s, const orc_settings* st, const uint8_t* stance,
                        double* l, double* h, double* rho);

/* Qadd [N+1][nx][nx] = Jc' diag(rho_c,k) Jc (zero at k = 0); Jc [nc][nx]. */
void orc_contact_weight(const orc_shape* s, const double* Jc, const double* rho_c, double* Qadd);

/* Riccati factor of the x-update (once per solve).  Outputs:
 *   K [N][nu][nx], L [N][nu][nu] (lower Cholesky factor of H_k, upper part 0),
 *   s [N][nx] = P_{k+1} c_k, P [N+1][nx][nx] (may be NULL).
 * qx [nx] (may be NULL) is added to the state weight (joint-limit penalties),
 * Qadd [N+1][nx][nx] (may be NULL) to the state weight of each stage.
 * Returns ORC_OK or ORC_NOT_PD (at the first stage whose H_k is not PD). */
int orc_factor(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
               const double* c, const double* q, const double* r, const double* rho,
               double mu, double* K, double* L, double* sv, double* P, const double* qx,
               const double* Qadd);

/* One x-update: given the linear terms qt [N+1][nx] and rt [N][nu], run the
 * back-sweep and the forward rollout from x0.  Outputs xt [N+1][nx], ut [N][nu]. */
void orc_xupdate(const orc_shape* s, const double* A, const double* B, const double* c,
                 const double* K, const double* L, const double* sv, const double* x0,
                 const double* qt, const double* rt, double* xt, double* ut);

/* KKT residuals of (x, u, z, y): res = {primal, dual, dynamics, complementarity}
 * (infinity norms) and the objective.  Costates come from the adjoint sweep. */
void orc_residuals(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
                   const double* c, const double* q, const double* r, const double* x_ref,
                   const double* u_ref, const double* x0, const double* tau_max, double mu,
                   const uint8_t* stance, const double* x, const double* u, const double* z,
                   const double* y, double* res, double* objective, const double* x_lo,
                   const double* x_hi, const double* zx, const double* yx, const double* Jc,
                   const double* zc, const double* yc);

/* Solve one agent.
 *   warm == 0: u, z, y start at 0; warm == 1: u, z, y are read from the
 *   buffers (previous solution).  x is always re-rolled from x0 and u.
 *   iters > 0: exactly that many iterations.
 *   iters <= 0: converge mode (tol, max_iters) -- used by tests only.
 * Outputs x [N+1][nx], u [N][nu], z [N][m], y [N][m], res[4], objective.
 * Joint limits (x_lo, x_hi [nx], may be NULL): the state rows' iterate
 * z_x, y_x [N][nx] (stages 1..N) is read on warm start and written.
 * No-slip rows (Jc [n_feet*foot_dim][nx], may be NULL): likewise z_c, y_c
 * [N][n_feet*foot_dim].
 * Returns a status code; *iters_done receives the iteration count. */
int orc_solve(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
              const double* c, const double* q, const double* r, const double* x_ref,
              const double* u_ref, const double* x0, const double* tau_max, double mu,
              const uint8_t* stance, int iters, int warm, double tol, int max_iters,
              double* x, double* u, double* z, double* y, double* res, double* objective,
              int* iters_done, const double* x_lo, const double* x_hi, double* zx, double* yx,
              const double* Jc, double* zc, double* yc);

/* Batched solve over agents with concatenated per-agent arrays (agent order),
 * OpenMP-parallel over agents.  shapes is [n][6] int32 (N,nx,nu,n_tau,n_feet,
 * foot_dim).  u_ref may be NULL.  res is [n][4], objective/status [n].
 * Returns the number of threads used. */
int orc_solve_batch(int32_t n, const int32_t* shapes, const orc_settings* st,
                    const double* A, const double* B, const double* c, const double* q,
                    const double* r, const double* x_ref, const double* u_ref,
                    const double* x0, const double* tau_max, const double* mu,
                    const uint8_t* stance, int iters, int warm, double* x, double* u,
                    double* z, double* y, double* res, double* objective, int32_t* status,
                    int n_threads, const double* x_lo, const double* x_hi, double* zx,
                    double* yx, const double* Jc, double* zc, double* yc);

/* Closed-loop state advance of the agents' own dynamics:
 * x0_next = A_0 x0 + B_0 u_0 + c_0 + noise (all [n] agents, concatenated). */
void orc_advance_batch(int32_t n, const int32_t* shapes, const double* A, const double* B,
                       const double* c, const double* x0, const double* u, const double* noise,
                       double* x0_next);

#ifdef __cplusplus
}
#endif
#endif
