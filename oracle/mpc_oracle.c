/*
 * FP64 CPU oracle for the batched MPC QP solve -- TEST INFRASTRUCTURE ONLY.
 * (Loaded by tests, the smoke check and the benchmark's CPU-baseline leg;
 * never by the product path.)  Plain loops, no blocking, no fusion: each
 * function follows the definition it cites so it can be checked by eye.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *   - cost in 1/2-form, no dt factor, terminal weight equal to Q, no x_0 term;
 *   - OSQP constants rho = 0.1, sigma = 1e-6, alpha = 1.6, equality rows get
 *     1e3 * rho, rows with both bounds infinite get rho_min = 1e-6;
 *   - dynamics rows kept exact (the rho_eq -> infinity limit of the
 *     quasi-definite system Eq. (kkt_system)), so every x-update is an
 *     equality-constrained LQR solved by a Riccati factor/sweep pair;
 *   - sigma applied to states and inputs; x_0 is pinned to xbar0;
 *   - cold start u = z = y = 0 with x rolled out from xbar0; warm start
 *     re-uses (u, z, y) and re-rolls x;
 *   - joint limits of Eq. (mpc_formulation), optional: a box
 *     x_lo <= x_k <= x_hi on every state component at stages 1..N (bounds
 *     per agent, the same at every stage; components without limits carry
 *     infinite bounds), split like the input rows with their own (z_x, y_x)
 *     and OSQP's penalty rule; since the rows are the identity on x, they add
 *     diag(rho_x) to the state weight of the Riccati factor and
 *     y_x - rho_x z_x to the state's linear term;
 *   - no-slip rows of Eq. (mpc_formulation), optional: J_f v_k = 0 for every
 *     foot f in stance, as rows Jc (n_feet * foot_dim rows over the whole
 *     state, zero on the positions; the Jacobian at the linearisation point,
 *     the same at every stage) on x_k, k = 1..N, with the stance of stage
 *     min(k, N-1) (x_N keeps the last stage's contacts); rows of a swinging
 *     foot are free.  Split like the input rows with their own (z_c, y_c) and
 *     OSQP's penalty rule, they add Jc' diag(rho_c,k) Jc to the state weight
 *     of stage k and Jc'(y_c - rho_c z_c) to the state's linear term.
 */
#include "mpc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t orc_rows(const orc_shape* s) { return s->nu + 4 * s->n_feet; }

/* C_k = [ I_nu ; Pi ]: the identity rows bound every input entry (torque box,
 * wrench components); Pi holds, per foot, the four facets of the friction
 * pyramid that linearises the contact cone of Eq. (mpc_formulation):
 *   f_x - mu f_z, -f_x - mu f_z, f_y - mu f_z, -f_y - mu f_z  (all <= 0 in stance). */
void orc_constraint_matrix(const orc_shape* s, double mu, double* C) {
  const int m = orc_rows(s), nu = s->nu;
  memset(C, 0, sizeof(double) * (size_t)m * nu);
  for (int i = 0; i < nu; ++i) C[i * nu + i] = 1.0;
  for (int f = 0; f < s->n_feet; ++f) {
    const int fx = s->n_tau + f * s->foot_dim, fy = fx + 1, fz = fx + 2;
    const int p = nu + 4 * f;
    C[(p + 0) * nu + fx] = 1.0;
    C[(p + 0) * nu + fz] = -mu;
    C[(p + 1) * nu + fx] = -1.0;
    C[(p + 1) * nu + fz] = -mu;
    C[(p + 2) * nu + fy] = 1.0;
    C[(p + 2) * nu + fz] = -mu;
    C[(p + 3) * nu + fy] = -1.0;
    C[(p + 3) * nu + fz] = -mu;
  }
}

/* Bounds of Eq. (mpc_formulation) (contact and swing rows) plus the torque
 * box, and OSQP's per-row penalty choice (equality rows stiffer, free rows
 * loose). */
void orc_stage_bounds(const orc_shape* s, const orc_settings* st, const double* tau_max,
                      const uint8_t* stance, double* l, double* h, double* rho) {
  const int m = orc_rows(s);
  for (int k = 0; k < s->N; ++k) {
    double* lk = l + (size_t)k * m;
    double* hk = h + (size_t)k * m;
    for (int i = 0; i < s->n_tau; ++i) {
      lk[i] = -tau_max[i];
      hk[i] = tau_max[i];
    }
    for (int f = 0; f < s->n_feet; ++f) {
      const int in_stance = stance[k * s->n_feet + f] != 0;
      for (int j = 0; j < s->foot_dim; ++j) {
        const int row = s->n_tau + f * s->foot_dim + j;
        if (in_stance) {
          lk[row] = (j == 2) ? 0.0 : -INFINITY; /* unilateral contact: f_z >= 0 */
          hk[row] = INFINITY;
        } else { /* swing foot: zero wrench */
          lk[row] = 0.0;
          hk[row] = 0.0;
        }
      }
      for (int j = 0; j < 4; ++j) {
        const int row = s->nu + 4 * f + j;
        lk[row] = -INFINITY;
        hk[row] = in_stance ? 0.0 : INFINITY;
      }
    }
    for (int i = 0; i < m; ++i) {
      double rr;
      if (lk[i] == hk[i])
        rr = st->rho_eq_scale * st->rho;
      else if (isinf(lk[i]) && isinf(hk[i]))
        rr = st->rho_min;
      else
        rr = st->rho;
      rho[(size_t)k * m + i] = rr;
    }
  }
}

/* Penalty of the state rows (joint limits): OSQP's rule applied to the box
 * x_lo <= x_k <= x_hi of every component. */
void orc_state_penalties(const orc_shape* s, const orc_settings* st, const double* x_lo,
                         const double* x_hi, double* rho_x) {
  for (int i = 0; i < s->nx; ++i) {
    if (x_lo[i] == x_hi[i])
      rho_x[i] = st->rho_eq_scale * st->rho;
    else if (isinf(x_lo[i]) && isinf(x_hi[i]))
      rho_x[i] = st->rho_min;
    else
      rho_x[i] = st->rho;
  }
}

int32_t orc_contact_rows(const orc_shape* s) { return s->n_feet * s->foot_dim; }

/* Bounds and penalties of the no-slip rows of x_k (k = 1..N, stored at k-1):
 * the foot_dim rows of foot f are J_f v_k = 0 (an equality row, penalty
 * rho_eq_scale * rho) while f is in stance at stage min(k, N-1), and free
 * (both bounds infinite, penalty rho_min) while it swings. */
void orc_contact_bounds(const orc_shape* s, const orc_settings* st, const uint8_t* stance,
                        double* l, double* h, double* rho) {
  const int nc = orc_contact_rows(s);
  for (int k = 1; k <= s->N; ++k) {
    const int sk = k < s->N ? k : s->N - 1;
    for (int f = 0; f < s->n_feet; ++f) {
      const int in_stance = stance[sk * s->n_feet + f] != 0;
      for (int j = 0; j < s->foot_dim; ++j) {
        const size_t idx = (size_t)(k - 1) * nc + f * s->foot_dim + j;
        l[idx] = in_stance ? 0.0 : -INFINITY;
        h[idx] = in_stance ? 0.0 : INFINITY;
        rho[idx] = in_stance ? st->rho_eq_scale * st->rho : st->rho_min;
      }
    }
  }
}

/* Qadd [N+1][nx][nx]: Jc' diag(rho_c,k) Jc for the no-slip rows of x_k,
 * k = 1..N, and zero at k = 0 (x_0 is fixed). */
void orc_contact_weight(const orc_shape* s, const double* Jc, const double* rho_c, double* Qadd) {
  const int nx = s->nx, nc = orc_contact_rows(s);
  memset(Qadd, 0, sizeof(double) * (size_t)(s->N + 1) * nx * nx);
  for (int k = 1; k <= s->N; ++k)
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        double acc = 0.0;
        for (int row = 0; row < nc; ++row)
          acc += Jc[row * nx + i] * rho_c[(size_t)(k - 1) * nc + row] * Jc[row * nx + j];
        Qadd[((size_t)k * nx + i) * nx + j] = acc;
      }
}

/* Lower Cholesky factor of the n x n SPD matrix H (row-major), row by row
 * (Cholesky-Banachiewicz).  Returns 0 if H is not positive definite. */
static int cholesky(int n, const double* H, double* L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double sum = H[i * n + j];
      for (int t = 0; t < j; ++t) sum -= L[i * n + t] * L[j * n + t];
      if (i == j) {
        if (!(sum > 0.0)) return 0;
        L[i * n + i] = sqrt(sum);
      } else {
        L[i * n + j] = sum / L[j * n + j];
      }
    }
  }
  return 1;
}

/* v <- (L L^T)^{-1} v by forward then backward substitution. */
static void chol_solve(int n, const double* L, double* v) {
  for (int i = 0; i < n; ++i) {
    double sum = v[i];
    for (int t = 0; t < i; ++t) sum -= L[i * n + t] * v[t];
    v[i] = sum / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double sum = v[i];
    for (int t = i + 1; t < n; ++t) sum -= L[t * n + i] * v[t];
    v[i] = sum / L[i * n + i];
  }
}

/* Riccati factor of the x-subproblem (the role of Eq. (ldl), once per solve).
 * P_N = Q~_N; for k = N-1 .. 0, with Q~_k = Q + sigma I (+ diag(rho_x) with
 * joint limits, + Qadd_k with no-slip rows):
 *   Rt_k = R + sigma I + C_k' diag(rho_k) C_k
 *   H_k = Rt_k + B_k' P_{k+1} B_k,   G_k = B_k' P_{k+1} A_k,   H_k = L_k L_k'
 *   K_k = -H_k^{-1} G_k,   s_k = P_{k+1} c_k
 *   P_k = Q~_k + A_k' P_{k+1} A_k + G_k' K_k   (then symmetrised)
 * qx (may be NULL): the joint-limit rows' penalties rho_x, added to Q~;
 * Qadd (may be NULL): [N+1][nx][nx], added to Q~_k (no-slip rows).          */
int orc_factor(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
               const double* c, const double* q, const double* r, const double* rho,
               double mu, double* K, double* L, double* sv, double* P, const double* qx,
               const double* Qadd) {
  const int N = s->N, nx = s->nx, nu = s->nu, m = orc_rows(s);
  double* C = (double*)malloc(sizeof(double) * m * nu);
  double* Pn = (double*)malloc(sizeof(double) * nx * nx);
  double* Pk = (double*)malloc(sizeof(double) * nx * nx);
  double* PA = (double*)malloc(sizeof(double) * nx * nx);
  double* PB = (double*)malloc(sizeof(double) * nx * nu);
  double* H = (double*)malloc(sizeof(double) * nu * nu);
  double* G = (double*)malloc(sizeof(double) * nu * nx);
  double* col = (double*)malloc(sizeof(double) * nu);
  int status = ORC_OK;
  orc_constraint_matrix(s, mu, C);

  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < nx; ++j)
      Pn[i * nx + j] = ((i == j) ? q[i] + st->sigma + (qx ? qx[i] : 0.0) : 0.0) +
                       (Qadd ? Qadd[((size_t)N * nx + i) * nx + j] : 0.0);
  if (P) memcpy(P + (size_t)N * nx * nx, Pn, sizeof(double) * nx * nx);

  for (int k = N - 1; k >= 0; --k) {
    const double* Ak = A + (size_t)k * nx * nx;
    const double* Bk = B + (size_t)k * nx * nu;
    const double* ck = c + (size_t)k * nx;
    const double* rk = rho + (size_t)k * m;
    double* Kk = K + (size_t)k * nu * nx;
    double* Lk = L + (size_t)k * nu * nu;

    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nu; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nx; ++t) acc += Pn[i * nx + t] * Bk[t * nu + j];
        PB[i * nu + j] = acc;
      }
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nx; ++t) acc += Pn[i * nx + t] * Ak[t * nx + j];
        PA[i * nx + j] = acc;
      }
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nu; ++j) {
        double acc = (i == j) ? r[i] + st->sigma : 0.0;
        for (int row = 0; row < m; ++row) acc += C[row * nu + i] * rk[row] * C[row * nu + j];
        for (int t = 0; t < nx; ++t) acc += Bk[t * nu + i] * PB[t * nu + j];
        H[i * nu + j] = acc;
      }
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nx; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nx; ++t) acc += Bk[t * nu + i] * PA[t * nx + j];
        G[i * nx + j] = acc;
      }
    for (int i = 0; i < nx; ++i) {
      double acc = 0.0;
      for (int t = 0; t < nx; ++t) acc += Pn[i * nx + t] * ck[t];
      sv[(size_t)k * nx + i] = acc;
    }
    if (!cholesky(nu, H, Lk)) {
      status = ORC_NOT_PD;
      break;
    }
    for (int j = 0; j < nx; ++j) {
      for (int i = 0; i < nu; ++i) col[i] = -G[i * nx + j];
      chol_solve(nu, Lk, col);
      for (int i = 0; i < nu; ++i) Kk[i * nx + j] = col[i];
    }
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        double acc = ((i == j) ? q[i] + st->sigma + (qx ? qx[i] : 0.0) : 0.0) +
                     (Qadd ? Qadd[((size_t)k * nx + i) * nx + j] : 0.0);
        for (int t = 0; t < nx; ++t) acc += Ak[t * nx + i] * PA[t * nx + j];
        for (int t = 0; t < nu; ++t) acc += G[t * nx + i] * Kk[t * nx + j];
        Pk[i * nx + j] = acc;
      }
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) Pn[i * nx + j] = 0.5 * (Pk[i * nx + j] + Pk[j * nx + i]);
    if (P) memcpy(P + (size_t)k * nx * nx, Pn, sizeof(double) * nx * nx);
  }
  free(C); free(Pn); free(Pk); free(PA); free(PB); free(H); free(G); free(col);
  return status;
}

/* One x-update (the role of Eqs. (backsolve_1)-(backsolve_2)).
 * Back-sweep, p_N = qt_N; for k = N-1 .. 0:
 *   p' = p_{k+1} + s_k,  h = rt_k + B_k' p',  d_k = -H_k^{-1} h,
 *   p_k = qt_k + A_k' p' + K_k' h.
 * Rollout, xt_0 = x0:  ut_k = K_k xt_k + d_k,  xt_{k+1} = A_k xt_k + B_k ut_k + c_k. */
void orc_xupdate(const orc_shape* s, const double* A, const double* B, const double* c,
                 const double* K, const double* L, const double* sv, const double* x0,
                 const double* qt, const double* rt, double* xt, double* ut) {
  const int N = s->N, nx = s->nx, nu = s->nu;
  double* p = (double*)malloc(sizeof(double) * nx);
  double* pp = (double*)malloc(sizeof(double) * nx);
  double* hv = (double*)malloc(sizeof(double) * nu);
  double* d = (double*)malloc(sizeof(double) * (size_t)N * nu);

  for (int i = 0; i < nx; ++i) p[i] = qt[(size_t)N * nx + i];
  for (int k = N - 1; k >= 0; --k) {
    const double* Ak = A + (size_t)k * nx * nx;
    const double* Bk = B + (size_t)k * nx * nu;
    const double* Kk = K + (size_t)k * nu * nx;
    for (int i = 0; i < nx; ++i) pp[i] = p[i] + sv[(size_t)k * nx + i];
    for (int j = 0; j < nu; ++j) {
      double acc = rt[(size_t)k * nu + j];
      for (int t = 0; t < nx; ++t) acc += Bk[t * nu + j] * pp[t];
      hv[j] = acc;
    }
    double* dk = d + (size_t)k * nu;
    for (int j = 0; j < nu; ++j) dk[j] = -hv[j];
    chol_solve(nu, L + (size_t)k * nu * nu, dk);
    for (int i = 0; i < nx; ++i) {
      double acc = qt[(size_t)k * nx + i];
      for (int t = 0; t < nx; ++t) acc += Ak[t * nx + i] * pp[t];
      for (int t = 0; t < nu; ++t) acc += Kk[t * nx + i] * hv[t];
      p[i] = acc;
    }
  }
  for (int i = 0; i < nx; ++i) xt[i] = x0[i];
  for (int k = 0; k < N; ++k) {
    const double* Ak = A + (size_t)k * nx * nx;
    const double* Bk = B + (size_t)k * nx * nu;
    const double* Kk = K + (size_t)k * nu * nx;
    const double* xk = xt + (size_t)k * nx;
    double* uk = ut + (size_t)k * nu;
    for (int j = 0; j < nu; ++j) {
      double acc = d[(size_t)k * nu + j];
      for (int t = 0; t < nx; ++t) acc += Kk[j * nx + t] * xk[t];
      uk[j] = acc;
    }
    for (int i = 0; i < nx; ++i) {
      double acc = c[(size_t)k * nx + i];
      for (int t = 0; t < nx; ++t) acc += Ak[i * nx + t] * xk[t];
      for (int t = 0; t < nu; ++t) acc += Bk[i * nu + t] * uk[t];
      xt[(size_t)(k + 1) * nx + i] = acc;
    }
  }
  free(p); free(pp); free(hv); free(d);
}

static double maxabs(double a, double b) { return fabs(a) > b ? fabs(a) : b; }

/* Stationarity and feasibility of (x, u, z, y) for the QP above.  Costates of
 * the dynamics rows: lambda_N = Q (x_N - r_N), lambda_k = Q (x_k - r_k) +
 * A_k' lambda_{k+1}, which zero the gradient in x_1..x_N by construction.
 *   res[0] primal   max |C_k u_k - z_k|
 *   res[1] dual     max |R (u_k - ubar_k) + B_k' lambda_{k+1} + C_k' y_k|
 *   res[2] dynamics max |x_{k+1} - A_k x_k - B_k u_k - c_k|, |x_0 - xbar0|
 *   res[3] complementarity / bounds: y_i > 0 needs z_i = h_i, y_i < 0 needs
 *          z_i = l_i (y in the normal cone of [l, h] at z), and l <= z <= h.
 * With joint limits (x_lo != NULL) the state rows join: their multipliers y_x
 * enter the costates, lambda_k = Q (x_k - r_k) + y_x,k + A_k' lambda_{k+1},
 * |x_k - z_x,k| the primal residual and (z_x, y_x) the complementarity test.
 * No-slip rows (Jc != NULL) likewise: Jc' y_c,k joins lambda_k, |Jc x_k - z_c,k|
 * the primal residual and (z_c, y_c) the complementarity test. */
static void complementarity(double lo, double hi, double zz, double yy, double* rc);

void orc_residuals(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
                   const double* c, const double* q, const double* r, const double* x_ref,
                   const double* u_ref, const double* x0, const double* tau_max, double mu,
                   const uint8_t* stance, const double* x, const double* u, const double* z,
                   const double* y, double* res, double* objective, const double* x_lo,
                   const double* x_hi, const double* zx, const double* yx, const double* Jc,
                   const double* zc, const double* yc) {
  const int N = s->N, nx = s->nx, nu = s->nu, m = orc_rows(s), nc = orc_contact_rows(s);
  double* lam = (double*)malloc(sizeof(double) * (size_t)(N + 1) * nx);
  double* lc = (double*)malloc(sizeof(double) * (size_t)N * (nc > 0 ? nc : 1));
  double* hc = (double*)malloc(sizeof(double) * (size_t)N * (nc > 0 ? nc : 1));
  double* rc_pen = (double*)malloc(sizeof(double) * (size_t)N * (nc > 0 ? nc : 1));
  if (Jc) orc_contact_bounds(s, st, stance, lc, hc, rc_pen);
  double* C = (double*)malloc(sizeof(double) * m * nu);
  double* l = (double*)malloc(sizeof(double) * (size_t)N * m);
  double* h = (double*)malloc(sizeof(double) * (size_t)N * m);
  double* rho = (double*)malloc(sizeof(double) * (size_t)N * m);
  orc_constraint_matrix(s, mu, C);
  orc_stage_bounds(s, st, tau_max, stance, l, h, rho);

  double obj = 0.0;
  for (int k = 1; k <= N; ++k)
    for (int i = 0; i < nx; ++i) {
      const double e = x[(size_t)k * nx + i] - x_ref[(size_t)k * nx + i];
      obj += 0.5 * q[i] * e * e;
    }
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < nu; ++j) {
      const double e = u[(size_t)k * nu + j] - (u_ref ? u_ref[(size_t)k * nu + j] : 0.0);
      obj += 0.5 * r[j] * e * e;
    }
  *objective = obj;

  for (int i = 0; i < nx; ++i) {
    double acc = q[i] * (x[(size_t)N * nx + i] - x_ref[(size_t)N * nx + i]) +
                 (x_lo ? yx[(size_t)(N - 1) * nx + i] : 0.0);
    if (Jc)
      for (int row = 0; row < nc; ++row) acc += Jc[row * nx + i] * yc[(size_t)(N - 1) * nc + row];
    lam[(size_t)N * nx + i] = acc;
  }
  for (int k = N - 1; k >= 1; --k) {
    const double* Ak = A + (size_t)k * nx * nx;
    for (int i = 0; i < nx; ++i) {
      double acc = q[i] * (x[(size_t)k * nx + i] - x_ref[(size_t)k * nx + i]);
      if (x_lo) acc += yx[(size_t)(k - 1) * nx + i];
      if (Jc)
        for (int row = 0; row < nc; ++row) acc += Jc[row * nx + i] * yc[(size_t)(k - 1) * nc + row];
      for (int t = 0; t < nx; ++t) acc += Ak[t * nx + i] * lam[(size_t)(k + 1) * nx + t];
      lam[(size_t)k * nx + i] = acc;
    }
  }
  double rp = 0.0, rd = 0.0, ry = 0.0, rc = 0.0;
  for (int i = 0; i < nx; ++i) ry = maxabs(x[i] - x0[i], ry);
  for (int k = 0; k < N; ++k) {
    const double* Ak = A + (size_t)k * nx * nx;
    const double* Bk = B + (size_t)k * nx * nu;
    const double* uk = u + (size_t)k * nu;
    const double* zk = z + (size_t)k * m;
    const double* yk = y + (size_t)k * m;
    for (int row = 0; row < m; ++row) {
      double acc = 0.0;
      for (int j = 0; j < nu; ++j) acc += C[row * nu + j] * uk[j];
      rp = maxabs(acc - zk[row], rp);
    }
    for (int j = 0; j < nu; ++j) {
      double acc = r[j] * (uk[j] - (u_ref ? u_ref[(size_t)k * nu + j] : 0.0));
      for (int t = 0; t < nx; ++t) acc += Bk[t * nu + j] * lam[(size_t)(k + 1) * nx + t];
      for (int row = 0; row < m; ++row) acc += C[row * nu + j] * yk[row];
      rd = maxabs(acc, rd);
    }
    for (int i = 0; i < nx; ++i) {
      double acc = x[(size_t)(k + 1) * nx + i] - c[(size_t)k * nx + i];
      for (int t = 0; t < nx; ++t) acc -= Ak[i * nx + t] * x[(size_t)k * nx + t];
      for (int t = 0; t < nu; ++t) acc -= Bk[i * nu + t] * uk[t];
      ry = maxabs(acc, ry);
    }
    for (int row = 0; row < m; ++row)
      complementarity(l[(size_t)k * m + row], h[(size_t)k * m + row], zk[row], yk[row], &rc);
    if (x_lo)  /* the state rows of x_{k+1} */
      for (int i = 0; i < nx; ++i) {
        const size_t idx = (size_t)k * nx + i;
        rp = maxabs(x[(size_t)(k + 1) * nx + i] - zx[idx], rp);
        complementarity(x_lo[i], x_hi[i], zx[idx], yx[idx], &rc);
      }
    if (Jc)  /* the no-slip rows of x_{k+1} */
      for (int row = 0; row < nc; ++row) {
        const size_t idx = (size_t)k * nc + row;
        double acc = 0.0;
        for (int t = 0; t < nx; ++t) acc += Jc[row * nx + t] * x[(size_t)(k + 1) * nx + t];
        rp = maxabs(acc - zc[idx], rp);
        complementarity(lc[idx], hc[idx], zc[idx], yc[idx], &rc);
      }
  }
  res[0] = rp;
  res[1] = rd;
  res[2] = ry;
  res[3] = rc;
  free(lam); free(C); free(l); free(h); free(rho); free(lc); free(hc); free(rc_pen);
}

/* Complementarity test of one row: y > 0 needs z = h, y < 0 needs z = l, and
 * l <= z <= h; the largest violation goes to *rc. */
static void complementarity(double lo, double hi, double zz, double yy, double* rc) {
  const double yp = yy > 0.0 ? yy : 0.0, ym = yy < 0.0 ? -yy : 0.0;
  const double a = isinf(hi) ? yp : fmin(yp, hi - zz);
  const double b = isinf(lo) ? ym : fmin(ym, zz - lo);
  *rc = maxabs(a, *rc);
  *rc = maxabs(b, *rc);
  if (zz > hi) *rc = maxabs(zz - hi, *rc);
  if (zz < lo) *rc = maxabs(lo - zz, *rc);
}

static int all_finite(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

static void fill_nan(double* v, size_t n) {
  for (size_t i = 0; i < n; ++i) v[i] = NAN;
}

int orc_solve(const orc_shape* s, const orc_settings* st, const double* A, const double* B,
              const double* c, const double* q, const double* r, const double* x_ref,
              const double* u_ref, const double* x0, const double* tau_max, double mu,
              const uint8_t* stance, int iters, int warm, double tol, int max_iters,
              double* x, double* u, double* z, double* y, double* res, double* objective,
              int* iters_done, const double* x_lo, const double* x_hi, double* zx, double* yx,
              const double* Jc, double* zc, double* yc) {
  const int N = s->N, nx = s->nx, nu = s->nu, m = orc_rows(s), nc = orc_contact_rows(s);
  const size_t nZx = (size_t)N * nx, nZc = (size_t)N * nc;
  const double alpha = st->alpha, sigma = st->sigma;
  const size_t nX = (size_t)(N + 1) * nx, nU = (size_t)N * nu, nZ = (size_t)N * m;
  int status = ORC_OK, it = 0;
  *iters_done = 0;

  const int finite_in = all_finite(A, (size_t)N * nx * nx) && all_finite(B, (size_t)N * nx * nu) &&
                        all_finite(c, (size_t)N * nx) && all_finite(q, nx) && all_finite(r, nu) &&
                        all_finite(x_ref, nX) && all_finite(x0, nx) &&
                        all_finite(tau_max, s->n_tau) && isfinite(mu) &&
                        (!u_ref || all_finite(u_ref, nU)) &&
                        (!warm || (all_finite(u, nU) && all_finite(z, nZ) && all_finite(y, nZ))) &&
                        (!x_lo || !warm || (all_finite(zx, nZx) && all_finite(yx, nZx))) &&
                        (!Jc || all_finite(Jc, (size_t)nc * nx)) &&
                        (!Jc || !warm || (all_finite(zc, nZc) && all_finite(yc, nZc)));
  int bounds_ok = 1;
  if (x_lo)
    for (int i = 0; i < nx; ++i)
      bounds_ok &= !isnan(x_lo[i]) && !isnan(x_hi[i]) && x_lo[i] <= x_hi[i];
  if (!finite_in || !bounds_ok) {
    fill_nan(x, nX); fill_nan(u, nU); fill_nan(z, nZ); fill_nan(y, nZ);
    if (x_lo) { fill_nan(zx, nZx); fill_nan(yx, nZx); }
    if (Jc) { fill_nan(zc, nZc); fill_nan(yc, nZc); }
    fill_nan(res, 4); *objective = NAN;
    return ORC_NONFINITE;
  }

  double* C = (double*)malloc(sizeof(double) * m * nu);
  double* l = (double*)malloc(sizeof(double) * nZ);
  double* h = (double*)malloc(sizeof(double) * nZ);
  double* rho = (double*)malloc(sizeof(double) * nZ);
  double* K = (double*)malloc(sizeof(double) * (size_t)N * nu * nx);
  double* L = (double*)malloc(sizeof(double) * (size_t)N * nu * nu);
  double* sv = (double*)malloc(sizeof(double) * (size_t)N * nx);
  double* qt = (double*)malloc(sizeof(double) * nX);
  double* rt = (double*)malloc(sizeof(double) * nU);
  double* xt = (double*)malloc(sizeof(double) * nX);
  double* ut = (double*)malloc(sizeof(double) * nU);
  double* rho_x = (double*)malloc(sizeof(double) * (size_t)nx);
  double* lc = (double*)malloc(sizeof(double) * (nZc > 0 ? nZc : 1));
  double* hc = (double*)malloc(sizeof(double) * (nZc > 0 ? nZc : 1));
  double* rho_c = (double*)malloc(sizeof(double) * (nZc > 0 ? nZc : 1));
  double* Qadd = Jc ? (double*)malloc(sizeof(double) * (size_t)(N + 1) * nx * nx) : NULL;
  orc_constraint_matrix(s, mu, C);
  orc_stage_bounds(s, st, tau_max, stance, l, h, rho);
  if (x_lo) orc_state_penalties(s, st, x_lo, x_hi, rho_x);
  if (Jc) {
    orc_contact_bounds(s, st, stance, lc, hc, rho_c);
    orc_contact_weight(s, Jc, rho_c, Qadd);
  }

  if (orc_factor(s, st, A, B, c, q, r, rho, mu, K, L, sv, NULL, x_lo ? rho_x : NULL, Qadd) != ORC_OK) {
    status = ORC_NOT_PD;
    goto done;
  }

  if (!warm) {
    memset(u, 0, sizeof(double) * nU);
    memset(z, 0, sizeof(double) * nZ);
    memset(y, 0, sizeof(double) * nZ);
    if (x_lo) {
      memset(zx, 0, sizeof(double) * nZx);
      memset(yx, 0, sizeof(double) * nZx);
    }
    if (Jc) {
      memset(zc, 0, sizeof(double) * nZc);
      memset(yc, 0, sizeof(double) * nZc);
    }
  }
  /* x^0: rollout of the dynamics from xbar0 under u^0 */
  for (int i = 0; i < nx; ++i) x[i] = x0[i];
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < nx; ++i) {
      double acc = c[(size_t)k * nx + i];
      for (int t = 0; t < nx; ++t) acc += A[(size_t)k * nx * nx + i * nx + t] * x[(size_t)k * nx + t];
      for (int t = 0; t < nu; ++t) acc += B[(size_t)k * nx * nu + i * nu + t] * u[(size_t)k * nu + t];
      x[(size_t)(k + 1) * nx + i] = acc;
    }

  const int limit = iters > 0 ? iters : max_iters;
  for (it = 0; it < limit; ++it) {
    /* linear terms of the x-subproblem (right-hand side of Eq. (kkt_system)) */
    for (int k = 0; k <= N; ++k)
      for (int i = 0; i < nx; ++i) {
        double acc = -q[i] * x_ref[(size_t)k * nx + i] - sigma * x[(size_t)k * nx + i];
        if (x_lo && k >= 1) acc += yx[(size_t)(k - 1) * nx + i] - rho_x[i] * zx[(size_t)(k - 1) * nx + i];
        if (Jc && k >= 1)
          for (int row = 0; row < nc; ++row) {
            const size_t idx = (size_t)(k - 1) * nc + row;
            acc += Jc[row * nx + i] * (yc[idx] - rho_c[idx] * zc[idx]);
          }
        qt[(size_t)k * nx + i] = acc;
      }
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < nu; ++j) {
        double acc = -sigma * u[(size_t)k * nu + j];
        if (u_ref) acc -= r[j] * u_ref[(size_t)k * nu + j];
        for (int row = 0; row < m; ++row)
          acc += C[row * nu + j] * (y[(size_t)k * m + row] - rho[(size_t)k * m + row] * z[(size_t)k * m + row]);
        rt[(size_t)k * nu + j] = acc;
      }
    orc_xupdate(s, A, B, c, K, L, sv, x0, qt, rt, xt, ut);
    /* relaxation, projection onto [l, h] and dual update (OSQP) */
    for (size_t i = 0; i < nX; ++i) x[i] = alpha * xt[i] + (1.0 - alpha) * x[i];
    for (int i = 0; i < nx; ++i) x[i] = x0[i];
    for (size_t i = 0; i < nU; ++i) u[i] = alpha * ut[i] + (1.0 - alpha) * u[i];
    for (int k = 0; k < N; ++k)
      for (int row = 0; row < m; ++row) {
        double zeta = 0.0;
        for (int j = 0; j < nu; ++j) zeta += C[row * nu + j] * ut[(size_t)k * nu + j];
        const size_t idx = (size_t)k * m + row;
        const double w = alpha * zeta + (1.0 - alpha) * z[idx];
        const double zn = fmin(fmax(w + y[idx] / rho[idx], l[idx]), h[idx]);
        y[idx] = y[idx] + rho[idx] * (w - zn);
        z[idx] = zn;
      }
    if (x_lo)  /* the state rows: zeta = xt_k, k = 1..N */
      for (int k = 1; k <= N; ++k)
        for (int i = 0; i < nx; ++i) {
          const size_t idx = (size_t)(k - 1) * nx + i;
          const double w = alpha * xt[(size_t)k * nx + i] + (1.0 - alpha) * zx[idx];
          const double zn = fmin(fmax(w + yx[idx] / rho_x[i], x_lo[i]), x_hi[i]);
          yx[idx] = yx[idx] + rho_x[i] * (w - zn);
          zx[idx] = zn;
        }
    if (Jc)  /* the no-slip rows: zeta = Jc xt_k, k = 1..N */
      for (int k = 1; k <= N; ++k)
        for (int row = 0; row < nc; ++row) {
          const size_t idx = (size_t)(k - 1) * nc + row;
          double zeta = 0.0;
          for (int t = 0; t < nx; ++t) zeta += Jc[row * nx + t] * xt[(size_t)k * nx + t];
          const double w = alpha * zeta + (1.0 - alpha) * zc[idx];
          const double zn = fmin(fmax(w + yc[idx] / rho_c[idx], lc[idx]), hc[idx]);
          yc[idx] = yc[idx] + rho_c[idx] * (w - zn);
          zc[idx] = zn;
        }
    if (iters <= 0) {
      double obj;
      orc_residuals(s, st, A, B, c, q, r, x_ref, u_ref, x0, tau_max, mu, stance, x, u, z, y,
                    res, &obj, x_lo, x_hi, zx, yx, Jc, zc, yc);
      double su = 1.0, sd = 1.0;
      for (int k = 0; k < N; ++k)
        for (int row = 0; row < m; ++row) {
          su = maxabs(z[(size_t)k * m + row], su);
          sd = maxabs(y[(size_t)k * m + row], sd);
        }
      for (size_t i = 0; i < nU; ++i) su = maxabs(u[i], su);
      if (x_lo)
        for (size_t i = 0; i < nZx; ++i) {
          su = maxabs(zx[i], su);
          sd = maxabs(yx[i], sd);
        }
      if (Jc)
        for (size_t i = 0; i < nZc; ++i) {
          su = maxabs(zc[i], su);
          sd = maxabs(yc[i], sd);
        }
      if (res[0] <= tol * su && res[1] <= tol * sd) {
        ++it;
        status = ORC_CONVERGED;
        break;
      }
    }
  }
  *iters_done = it;
  orc_residuals(s, st, A, B, c, q, r, x_ref, u_ref, x0, tau_max, mu, stance, x, u, z, y, res,
                objective, x_lo, x_hi, zx, yx, Jc, zc, yc);
  if (!(all_finite(x, nX) && all_finite(u, nU) && all_finite(z, nZ) && all_finite(y, nZ)) ||
      (x_lo && !(all_finite(zx, nZx) && all_finite(yx, nZx))) ||
      (Jc && !(all_finite(zc, nZc) && all_finite(yc, nZc))))
    status = ORC_NONFINITE;

done:
  if (status == ORC_NOT_PD || status == ORC_NONFINITE) {
    fill_nan(x, nX); fill_nan(u, nU); fill_nan(z, nZ); fill_nan(y, nZ);
    if (x_lo) { fill_nan(zx, nZx); fill_nan(yx, nZx); }
    if (Jc) { fill_nan(zc, nZc); fill_nan(yc, nZc); }
    fill_nan(res, 4); *objective = NAN;
  }
  free(C); free(l); free(h); free(rho); free(K); free(L); free(sv);
  free(qt); free(rt); free(xt); free(ut); free(rho_x); free(lc); free(hc); free(rho_c); free(Qadd);
  return status;
}

typedef struct {
  size_t A, B, c, q, r, xr, x0, tau, st, x, u, z, J, zc;
} offs;

static void agent_offsets(int32_t n, const int32_t* shapes, offs* o) {
  offs cur;
  memset(&cur, 0, sizeof(cur));
  for (int32_t a = 0; a < n; ++a) {
    o[a] = cur;
    const int32_t* sh = shapes + 6 * a;
    const size_t N = sh[0], nx = sh[1], nu = sh[2], nt = sh[3], nf = sh[4];
    const size_t m = nu + 4 * nf;
    cur.A += N * nx * nx;
    cur.B += N * nx * nu;
    cur.c += N * nx;
    cur.q += nx;
    cur.r += nu;
    cur.xr += (N + 1) * nx;
    cur.x0 += nx;
    cur.tau += nt;
    cur.st += N * nf;
    cur.x += (N + 1) * nx;
    cur.u += N * nu;
    cur.z += N * m;
    cur.J += nf * (size_t)sh[5] * nx;
    cur.zc += N * nf * (size_t)sh[5];
  }
}

int orc_solve_batch(int32_t n, const int32_t* shapes, const orc_settings* st,
                    const double* A, const double* B, const double* c, const double* q,
                    const double* r, const double* x_ref, const double* u_ref,
                    const double* x0, const double* tau_max, const double* mu,
                    const uint8_t* stance, int iters, int warm, double* x, double* u,
                    double* z, double* y, double* res, double* objective, int32_t* status,
                    int n_threads, const double* x_lo, const double* x_hi, double* zx,
                    double* yx, const double* Jc, double* zc, double* yc) {
  offs* o = (offs*)malloc(sizeof(offs) * (n > 0 ? n : 1));
  agent_offsets(n, shapes, o);
  int used = 1;
#ifdef _OPENMP
  if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
  for (int32_t a = 0; a < n; ++a) {
    const int32_t* sh = shapes + 6 * a;
    orc_shape s = {sh[0], sh[1], sh[2], sh[3], sh[4], sh[5]};
    int done_it;
    status[a] = orc_solve(&s, st, A + o[a].A, B + o[a].B, c + o[a].c, q + o[a].q, r + o[a].r,
                          x_ref + o[a].xr, u_ref ? u_ref + o[a].u : NULL, x0 + o[a].x0,
                          tau_max + o[a].tau, mu[a], stance + o[a].st, iters, warm, 0.0, 0,
                          x + o[a].x, u + o[a].u, z + o[a].z, y + o[a].z, res + 4 * (size_t)a,
                          objective + a, &done_it, x_lo ? x_lo + o[a].q : NULL,
                          x_lo ? x_hi + o[a].q : NULL, x_lo ? zx + o[a].c : NULL,
                          x_lo ? yx + o[a].c : NULL, Jc ? Jc + o[a].J : NULL,
                          Jc ? zc + o[a].zc : NULL, Jc ? yc + o[a].zc : NULL);
  }
#ifdef _OPENMP
  used = n_threads;
#endif
  free(o);
  return used;
}

void orc_advance_batch(int32_t n, const int32_t* shapes, const double* A, const double* B,
                       const double* c, const double* x0, const double* u, const double* noise,
                       double* x0_next) {
  offs* o = (offs*)malloc(sizeof(offs) * (n > 0 ? n : 1));
  agent_offsets(n, shapes, o);
  for (int32_t a = 0; a < n; ++a) {
    const int nx = shapes[6 * a + 1], nu = shapes[6 * a + 2];
    const double* A0 = A + o[a].A;
    const double* B0 = B + o[a].B;
    for (int i = 0; i < nx; ++i) {
      double acc = c[o[a].c + i] + noise[o[a].x0 + i];
      for (int t = 0; t < nx; ++t) acc += A0[i * nx + t] * x0[o[a].x0 + t];
      for (int t = 0; t < nu; ++t) acc += B0[i * nu + t] * u[o[a].u + t];
      x0_next[o[a].x0 + i] = acc;
    }
  }
  free(o);
}
