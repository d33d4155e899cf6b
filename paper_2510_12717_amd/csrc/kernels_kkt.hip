// The paper's own inner solve on the GPU: OSQP on the standard form with the
// dynamics as equality rows (finite rho_eq = rho_eq_scale * rho), the
// quasi-definite KKT matrix of Eq. (kkt_system) factored once per solve
// (Eq. (ldl)) and every iteration's system solved by substitution
// (Eqs. (backsolve_1)-(backsolve_2)).  One workgroup per agent, any shape within
// the plan limits, FP64 arithmetic for every io type.
//
// Unknowns v = (x_1 .. x_N, u_0 .. u_{N-1}) (x_0 = xbar0 substituted into the
// first dynamics row), rows: dynamics of stage k, x_{k+1} - A_k x_k - B_k u_k
// in [c_k, c_k] (c_0 + A_0 xbar0 at k = 0), and the input rows C_k u_k.
//
// Elimination order of the LDL^T: every row's multiplier first (its pivot is
// -1/rho_i, and it couples only to the unknowns of its own row), which leaves
// the Schur complement R = P + sigma I + A' diag(rho) A on the primal
// unknowns; in the stage order w_k = (u_k, x_{k+1}) R is block tridiagonal:
//   D_k = [ Rt_k + rho_d B_k'B_k      -rho_d B_k'                            ]
//         [ -rho_d B_k                 Q + (sigma + rho_d) I + rho_d A_{k+1}'A_{k+1} ]
//   (Rt_k = R + sigma I + C_k' diag(rho_k) C_k; the A_{k+1} term for k < N-1)
//   E_k = R[w_k, w_{k-1}] = [rho_d B_k'A_k; -rho_d A_k] on the columns of x_k.
// Its block LDL^T in stage order: S_0 = D_0, S_k = D_k - E_k S_{k-1}^{-1} E_k',
// each S_k inverted in FP64 (Gauss-Jordan, SPD so no pivoting) and stored in
// the io type.
// A solve R w = b is then the forward sweep yh_k = b_k - E_k S_{k-1}^{-1} yh_{k-1}
// and the backward sweep w_k = S_k^{-1} (yh_k - E_{k+1}' w_{k+1}); the rows'
// values A xt follow from the primal solution (OSQP's zt = z + (nu - y)/rho
// equals A xt), so the multipliers' part of the solution is never formed.
//
// Iteration (relaxation alpha): xt from R xt = sigma v - q + A'(rho z - y),
// zt = A xt, v <- alpha xt + (1 - alpha) v, z+ = clip(alpha zt + (1 - alpha) z
// + y/rho, l, h), y <- y + rho (alpha zt + (1 - alpha) z - z+), z <- z+.
// Cold start: u = 0, x rolled out from xbar0, z = A v, y = 0; a warm start
// re-uses the resident x, u and both row blocks' z, y.
#include <math.h>

#include "generic_ops.h"
#include "mpc_internal.h"
#include "stage_rows.h"

#include <mutex>

namespace mpc {

namespace {

// Factor: S_k^{-1} of every stage, [N][nw][nw] per agent (io type) at ws + d.ows.
// The Schur correction of stage k is E_k M E_k' with M = [S_{k-1}^{-1}]_xx and
// E_k = [rho_d B_k' A_k; -rho_d A_k]: with Y = A_k M A_k' it is
//   [rho_d^2 B_k'Y B_k, -rho_d^2 B_k'Y; -rho_d^2 Y B_k, rho_d^2 Y].
// 1024 threads: one agent's factor fills a CU (its LDS allows no second one),
// and the stage work is element-parallel between barriers.
template <typename T>
__global__ void __launch_bounds__(1024)
k_kkt_factor(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
             Inputs<T> in, SolverConsts sc_all, T* __restrict__ ws, int32_t* __restrict__ status) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, a);
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m, nw = nu + nx;
  const int tid = threadIdx.x, nt = blockDim.x;
  using D = double;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  D* S = reinterpret_cast<D*>(smem_raw);  // S_k, inverted in place     nw*nw
  D* M = S + nw * nw;                     // [S_{k-1}^{-1}]_xx            nx*nx
  D* G = M + nx * nx;                     // A_k M, then A_{k+1}          nx*nx
  D* Y = G + nx * nx;                     // A_k M A_k'                   nx*nx
  D* Ab = Y + nx * nx;                    // A_k                          nx*nx
  D* W = Ab + nx * nx;                    // B_k' Y                       nu*nx
  D* Bb = W + nu * nx;                    // B_k                          nx*nu
  D* rhok = Bb + nx * nu;                 // row penalties of stage k     m
  __shared__ int s_flag;

  const T* A = in.A + d.oA;
  const T* B = in.B + d.oB;
  const T* q = in.q + d.oq;
  const T* r = in.r + d.orr;
  const T* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const D mu = (D)in.mu[d.omu];
  const D rd = sc.rho_eq * sc.rho;  // penalty of the dynamics rows (equalities)
  const D rd2 = rd * rd;
  T* Sinv = ws + d.ows;

  if (tid == 0) s_flag = 0;
  __syncthreads();
  bool ok = finite_all(A, (int64_t)N * nx * nx, tid, nt) && finite_all(B, (int64_t)N * nx * nu, tid, nt) &&
            finite_all(in.c + d.oc, (int64_t)N * nx, tid, nt) && finite_all(q, nx, tid, nt) &&
            finite_all(r, nu, tid, nt) && finite_all(in.xr + d.oxr, (int64_t)(N + 1) * nx, tid, nt) &&
            finite_all(in.x0 + d.ox0, nx, tid, nt) && finite_all(tau, d.n_tau, tid, nt) &&
            (bool)isfinite(mu) && (!in.uref || finite_all(in.uref + d.our, (int64_t)N * nu, tid, nt));
  if (!ok) atomicOr(&s_flag, 1);
  for (int idx = tid; idx < nx * nx; idx += nt) Ab[idx] = (D)A[idx];  // A_0
  __syncthreads();
  if (s_flag) {
    if (tid == 0) status[a] = AGENT_NONFINITE;
    return;
  }

  for (int k = 0; k < N; ++k) {
    const T* Bk = B + (int64_t)k * nx * nu;
    for (int idx = tid; idx < nx * nu; idx += nt) Bb[idx] = (D)Bk[idx];
    if (k >= 1) {
      // G = A_k M, Y = G A_k', W = B_k' Y
      for (int idx = tid; idx < nx * nx; idx += nt) {
        const int i = idx / nx, j = idx % nx;
        D acc = 0;
        for (int t = 0; t < nx; ++t) acc += Ab[i * nx + t] * M[t * nx + j];
        G[idx] = acc;
      }
      __syncthreads();
      for (int idx = tid; idx < nx * nx; idx += nt) {
        const int i = idx / nx, j = idx % nx;
        D acc = 0;
        for (int t = 0; t < nx; ++t) acc += G[i * nx + t] * Ab[j * nx + t];
        Y[idx] = acc;
      }
      __syncthreads();
      for (int idx = tid; idx < nu * nx; idx += nt) {
        const int i = idx / nx, j = idx % nx;
        D acc = 0;
        for (int t = 0; t < nx; ++t) acc += Bb[t * nu + i] * Y[t * nx + j];
        W[idx] = acc;
      }
    }
    __syncthreads();
    // A_{k+1} into G (dead now), the row penalties of stage k
    if (k + 1 < N) {
      const T* An = A + (int64_t)(k + 1) * nx * nx;
      for (int idx = tid; idx < nx * nx; idx += nt) G[idx] = (D)An[idx];
    }
    for (int i = tid; i < m; i += nt) {
      D lo, hi;
      row_bounds<D, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rhok[i]);
    }
    __syncthreads();
    // S = D_k - E_k M E_k'
    for (int idx = tid; idx < nw * nw; idx += nt) {
      const int i = idx / nw, j = idx % nw;
      D v = 0;
      if (i < nu && j < nu) {
        if (i == j) v = rtilde_diag<D, D>(d, j, (D)r[j], mu, rhok, sc);
        D acc = 0, cor = 0;
        for (int t = 0; t < nx; ++t) {
          acc += Bb[t * nu + i] * Bb[t * nu + j];
          if (k >= 1) cor += W[i * nx + t] * Bb[t * nu + j];
        }
        v += rd * acc - rd2 * cor;
      } else if (i < nu) {
        v = -rd * Bb[(j - nu) * nu + i] + (k >= 1 ? rd2 * W[i * nx + (j - nu)] : 0.0);
      } else if (j < nu) {
        v = -rd * Bb[(i - nu) * nu + j] + (k >= 1 ? rd2 * W[j * nx + (i - nu)] : 0.0);
      } else {
        const int ii = i - nu, jj = j - nu;
        if (ii == jj) v = (D)q[ii] + sc.sigma + rd;
        if (k + 1 < N) {
          D acc = 0;
          for (int t = 0; t < nx; ++t) acc += G[t * nx + ii] * G[t * nx + jj];
          v += rd * acc;
        }
        if (k >= 1) v -= rd2 * Y[ii * nx + jj];
      }
      S[idx] = v;
    }
    __syncthreads();
    // In-place Gauss-Jordan inverse of the SPD S (pivots on the diagonal)
    for (int p = 0; p < nw; ++p) {
      const D piv = S[p * nw + p];
      if (!(piv > 0.0)) {
        if (tid == 0) s_flag = 1;
      }
      __syncthreads();
      if (s_flag) break;
      const D ip = 1.0 / piv;
      // rows i != p, columns j != p: S_ij -= S_ip S_pj / S_pp (S_pj read before any write)
      for (int idx = tid; idx < nw * nw; idx += nt) {
        const int i = idx / nw, j = idx % nw;
        if (i != p && j != p) S[idx] -= S[i * nw + p] * S[p * nw + j] * ip;
      }
      __syncthreads();
      for (int t = tid; t < nw; t += nt) {
        if (t != p) {
          S[p * nw + t] *= ip;
          S[t * nw + p] *= -ip;
        }
      }
      __syncthreads();
      if (tid == 0) S[p * nw + p] = ip;
      __syncthreads();
    }
    if (s_flag) {
      if (tid == 0) status[a] = AGENT_NOT_PD;
      return;
    }
    for (int idx = tid; idx < nw * nw; idx += nt) Sinv[(int64_t)k * nw * nw + idx] = (T)S[idx];
    for (int idx = tid; idx < nx * nx; idx += nt) {
      const int i = idx / nx, j = idx % nx;
      M[idx] = S[(nu + i) * nw + nu + j];
      Ab[idx] = G[idx];  // A_{k+1} becomes the next stage's A_k
    }
    __syncthreads();
  }
  if (tid == 0) status[a] = AGENT_OK;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_kkt_admm(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
           Inputs<T> in, SolverConsts sc_all, int iters, int warm, const T* __restrict__ ws,
           State<T> st, T* __restrict__ gzd, T* __restrict__ gyd) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, a);
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m, nw = nu + nx;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* X = st.x + d.ox;
  T* U = st.u + d.ou;
  T* Z = st.z + d.oz;
  T* Y = st.y + d.oy;
  T* ZD = gzd + d.oc;
  T* YD = gyd + d.oc;
  if (st.status[a] != AGENT_OK) {
    const T nan = (T)NAN;
    for (int i = tid; i < (N + 1) * nx; i += nt) X[i] = nan;
    for (int i = tid; i < N * nu; i += nt) U[i] = nan;
    for (int i = tid; i < N * m; i += nt) {
      Z[i] = nan;
      Y[i] = nan;
    }
    for (int i = tid; i < N * nx; i += nt) {
      ZD[i] = nan;
      YD[i] = nan;
    }
    return;
  }
  using V = double;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* x = reinterpret_cast<V*>(smem_raw);  // (N+1)*nx, x_0 = xbar0
  V* u = x + (N + 1) * nx;                // N*nu
  V* z = u + N * nu;                      // N*m   input rows
  V* y = z + N * m;                       // N*m
  V* zd = y + N * m;                      // N*nx  dynamics rows
  V* yd = zd + N * nx;                    // N*nx
  V* b = yd + N * nx;                     // N*nw  right-hand side, then yh
  V* w = b + N * nw;                      // N*nw  solution (ut_k, xt_{k+1}); rho_d zd - yd first
  V* t = w + N * nw;                      // nx    [S_{k-1}^{-1} yh_{k-1}]_x, then B u - x
  V* av = t + nx;                         // nx    A_k t, then rho_d A_{k+1}'(B u - x)
  V* rhs0 = av + nx;                      // nx    c_0 + A_0 xbar0

  const T* A = in.A + d.oA;
  const T* B = in.B + d.oB;
  const T* c = in.c + d.oc;
  const T* q = in.q + d.oq;
  const T* r = in.r + d.orr;
  const T* xr = in.xr + d.oxr;
  const T* x0 = in.x0 + d.ox0;
  const T* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const T* uref = in.uref ? in.uref + d.our : nullptr;
  const V mu = (V)in.mu[d.omu];
  const V rd = sc.rho_eq * sc.rho;
  const T* Sinv = ws + d.ows;
  const V sigma = sc.sigma, alpha = sc.alpha, oma = 1.0 - sc.alpha;

  const bool wm = agent_warm(warm, d);
  for (int i = tid; i < nx; i += nt) x[i] = (V)x0[i];
  for (int i = tid; i < N * nu; i += nt) u[i] = wm ? (V)U[i] : 0.0;
  for (int i = tid; i < N * m; i += nt) {
    z[i] = wm ? (V)Z[i] : 0.0;
    y[i] = wm ? (V)Y[i] : 0.0;
  }
  if (wm)
    for (int i = tid; i < N * nx; i += nt) {
      x[nx + i] = (V)X[nx + i];
      zd[i] = (V)ZD[i];
      yd[i] = (V)YD[i];
    }
  __syncthreads();
  quad_matvec<V>(nx, nx, [&](int i, int tt) { return A[i * nx + tt]; }, x,
                 [&](int i, V acc) { rhs0[i] = (V)c[i] + acc; }, tid, nt);
  __syncthreads();
  if (!wm) {
    // x rolled out under u = 0; z = A v: the dynamics rows at their bounds
    for (int k = 0; k < N; ++k) {
      const T* Ak = A + (int64_t)k * nx * nx;
      quad_matvec<V>(nx, nx, [&](int i, int tt) { return Ak[i * nx + tt]; }, x + k * nx,
                     [&](int i, V acc) { x[(k + 1) * nx + i] = (V)c[(int64_t)k * nx + i] + acc; },
                     tid, nt);
      __syncthreads();
    }
    for (int i = tid; i < N * nx; i += nt) {
      zd[i] = i < nx ? rhs0[i] : (V)c[i];
      yd[i] = 0.0;
    }
    __syncthreads();
  }

  for (int it = 0; it < iters; ++it) {
    // w := rho_d zd - yd (the dynamics rows' part of A'(rho z - y))
    for (int i = tid; i < N * nx; i += nt) w[i] = rd * zd[i] - yd[i];
    __syncthreads();
    // b_u,k = sigma u_k + R ubar_k + C_k'(rho z_k - y_k) - B_k'(rho_d zd_k - yd_k)
    quad_dot<V>(N * nu, nx,
                [&](int idx, int tt) {
                  const int k = idx / nu, j = idx % nu;
                  return (V)B[((int64_t)k * nx + tt) * nu + j] * w[k * nx + tt];
                },
                [&](int idx, V acc) {
                  const int k = idx / nu, j = idx % nu;
                  const V* yk = y + k * m;
                  const V* zk = z + k * m;
                  const uint8_t* stk = stance + k * d.n_feet;
                  auto wr = [&](int i) {
                    V lo, hi, rr;
                    row_bounds<V, T>(d, i, stk, tau, sc, lo, hi, rr);
                    return rr * zk[i] - yk[i];
                  };
                  V v = wr(j);
                  if (j >= d.n_tau) {
                    const int f = (j - d.n_tau) / d.foot_dim, cc = (j - d.n_tau) % d.foot_dim;
                    const int b0 = nu + 4 * f;
                    if (cc == 0) v += wr(b0) - wr(b0 + 1);
                    if (cc == 1) v += wr(b0 + 2) - wr(b0 + 3);
                    if (cc == 2) v -= mu * (wr(b0) + wr(b0 + 1) + wr(b0 + 2) + wr(b0 + 3));
                  }
                  V bu = sigma * u[idx] + v - acc;
                  if (uref) bu += (V)r[j] * (V)uref[idx];
                  b[k * nw + j] = bu;
                },
                tid, nt);
    // b_x,k+1 = sigma x_{k+1} + Q r_{k+1} + (rho_d zd_k - yd_k) - A_{k+1}'(rho_d zd_{k+1} - yd_{k+1})
    quad_dot<V>(N * nx, nx,
                [&](int idx, int tt) {
                  const int k = idx / nx, i = idx % nx;
                  if (k + 1 >= N) return (V)0;
                  return (V)A[((int64_t)(k + 1) * nx + tt) * nx + i] * w[(k + 1) * nx + tt];
                },
                [&](int idx, V acc) {
                  const int k = idx / nx, i = idx % nx;
                  const int xi = (k + 1) * nx + i;
                  b[k * nw + nu + i] = sigma * x[xi] + (V)q[i] * (V)xr[xi] + w[idx] - acc;
                },
                tid, nt);
    __syncthreads();
    // forward sweep: yh_k = b_k - E_k t_{k-1}, t_k = [S_k^{-1} yh_k]_x
    for (int k = 0; k < N; ++k) {
      const T* Sk = Sinv + (int64_t)k * nw * nw;
      if (k >= 1) {
        const T* Ak = A + (int64_t)k * nx * nx;
        const T* Bk = B + (int64_t)k * nx * nu;
        quad_matvec<V>(nx, nx, [&](int i, int tt) { return Ak[i * nx + tt]; }, t,
                       [&](int i, V acc) { av[i] = acc; }, tid, nt);
        __syncthreads();
        // E_k t = [rho_d B_k' (A_k t); -rho_d A_k t]
        quad_dot<V>(nw, nx,
                    [&](int i, int tt) { return i < nu ? (V)Bk[tt * nu + i] * av[tt] : (V)0; },
                    [&](int i, V acc) {
                      b[k * nw + i] -= i < nu ? rd * acc : -rd * av[i - nu];
                    },
                    tid, nt);
        __syncthreads();
      }
      quad_matvec<V>(nx, nw, [&](int i, int tt) { return Sk[(nu + i) * nw + tt]; }, b + k * nw,
                     [&](int i, V acc) { t[i] = acc; }, tid, nt);
      __syncthreads();
    }
    // backward sweep: w_k = S_k^{-1} (yh_k - E_{k+1}' w_{k+1}),
    // E_{k+1}' w_{k+1} = rho_d A_{k+1}' (B_{k+1} ut_{k+1} - xt_{k+2}) on the rows of x_{k+1}
    for (int k = N - 1; k >= 0; --k) {
      if (k + 1 < N) {
        const T* An = A + (int64_t)(k + 1) * nx * nx;
        const T* Bn = B + (int64_t)(k + 1) * nx * nu;
        const V* wn = w + (k + 1) * nw;
        quad_matvec<V>(nx, nu, [&](int i, int tt) { return Bn[i * nu + tt]; }, wn,
                       [&](int i, V acc) { t[i] = acc - wn[nu + i]; }, tid, nt);
        __syncthreads();
        quad_matvec<V>(nx, nx, [&](int i, int tt) { return An[tt * nx + i]; }, t,
                       [&](int i, V acc) { b[k * nw + nu + i] -= rd * acc; }, tid, nt);
        __syncthreads();
      }
      const T* Sk = Sinv + (int64_t)k * nw * nw;
      quad_matvec<V>(nw, nw, [&](int i, int tt) { return Sk[i * nw + tt]; }, b + k * nw,
                     [&](int i, V acc) { w[k * nw + i] = acc; }, tid, nt);
      __syncthreads();
    }
    // zt = A vt and the OSQP updates.  Dynamics row k: xt_{k+1} - A_k xt_k - B_k ut_k
    // (xt_0 = 0: xbar0 sits in the bound); the rows are equalities, so z+ is the bound.
    quad_dot<V>(N * nx, nx + nu,
                [&](int idx, int tt) {
                  const int k = idx / nx, i = idx % nx;
                  if (tt < nx)
                    return k >= 1 ? (V)A[((int64_t)k * nx + i) * nx + tt] * w[(k - 1) * nw + nu + tt] : (V)0;
                  const int j = tt - nx;
                  return (V)B[((int64_t)k * nx + i) * nu + j] * w[k * nw + j];
                },
                [&](int idx, V acc) {
                  const int k = idx / nx, i = idx % nx;
                  const V zt = w[k * nw + nu + i] - acc;
                  const V wv = alpha * zt + oma * zd[idx];
                  const V zn = k == 0 ? rhs0[i] : (V)c[idx];
                  yd[idx] = yd[idx] + rd * (wv - zn);
                  zd[idx] = zn;
                },
                tid, nt);
    for (int idx = tid; idx < N * m; idx += nt) {
      const int k = idx / m, i = idx % m;
      V lo, hi, rr;
      row_bounds<V, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rr);
      const V zt = c_row<V>(d, i, mu, w + k * nw);
      const V wv = alpha * zt + oma * z[idx];
      const V zn = fmin(fmax(wv + y[idx] / rr, lo), hi);
      y[idx] = y[idx] + rr * (wv - zn);
      z[idx] = zn;
    }
    __syncthreads();
    for (int idx = tid; idx < N * nu; idx += nt) {
      const int k = idx / nu, j = idx % nu;
      u[idx] = alpha * w[k * nw + j] + oma * u[idx];
    }
    for (int idx = tid; idx < N * nx; idx += nt) {
      const int k = idx / nx, i = idx % nx;
      x[nx + idx] = alpha * w[k * nw + nu + i] + oma * x[nx + idx];
    }
    __syncthreads();
  }

  bool ok = true;
  for (int i = tid; i < (N + 1) * nx; i += nt) {
    X[i] = (T)x[i];
    ok &= (bool)isfinite(X[i]);
  }
  for (int i = tid; i < N * nu; i += nt) {
    U[i] = (T)u[i];
    ok &= (bool)isfinite(U[i]);
  }
  for (int i = tid; i < N * m; i += nt) {
    Z[i] = (T)z[i];
    Y[i] = (T)y[i];
    ok &= (bool)isfinite(Z[i]) && (bool)isfinite(Y[i]);
  }
  for (int i = tid; i < N * nx; i += nt) {
    ZD[i] = (T)zd[i];
    YD[i] = (T)yd[i];
    ok &= (bool)isfinite(ZD[i]) && (bool)isfinite(YD[i]);
  }
  if (!ok) st.status[a] = AGENT_NONFINITE;
}

}  // namespace

template <typename T>
hipError_t launch_kkt_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                             SolverConsts sc, T* ws, int32_t* status, size_t lds,
                             hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kkt_factor<T>, dim3(n_launch), dim3(1024), lds, stream, d_desc, list, n_launch,
                     in, sc, ws, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_kkt_admm(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                           SolverConsts sc, int iters, int warm, const T* ws, State<T> st,
                           T* zd, T* yd, size_t lds, hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kkt_admm<T>, dim3(n_launch), dim3(256), lds, stream, d_desc, list, n_launch,
                     in, sc, iters, warm, ws, st, zd, yd);
  return hipGetLastError();
}

hipError_t kkt_set_lds_limits(size_t lds_factor, size_t lds_admm) {
  static std::mutex mu;
  static size_t cur[2] = {0, 0};
  std::lock_guard<std::mutex> lock(mu);
  hipError_t e = hipSuccess;
#define MPC_SET(kern, bytes)                                                                  \
  if (e == hipSuccess)                                                                        \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes));
  if (lds_factor > cur[0]) {
    MPC_SET(k_kkt_factor<float>, lds_factor)
    MPC_SET(k_kkt_factor<double>, lds_factor)
    if (e == hipSuccess) cur[0] = lds_factor;
  }
  if (lds_admm > cur[1]) {
    MPC_SET(k_kkt_admm<float>, lds_admm)
    MPC_SET(k_kkt_admm<double>, lds_admm)
    if (e == hipSuccess) cur[1] = lds_admm;
  }
#undef MPC_SET
  return e;
}

#define MPC_INSTANTIATE(T)                                                                        \
  template hipError_t launch_kkt_factor<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,      \
                                           SolverConsts, T*, int32_t*, size_t, hipStream_t);      \
  template hipError_t launch_kkt_admm<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,        \
                                         SolverConsts, int, int, const T*, State<T>, T*, T*,      \
                                         size_t, hipStream_t);
MPC_INSTANTIATE(float)
MPC_INSTANTIATE(double)

}  // namespace mpc
