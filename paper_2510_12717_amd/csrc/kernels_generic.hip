// Generic kernels of the batched MPC solve: one workgroup per agent, any shape
// within the plan limits, templated on the arithmetic type (double or float).
//
//   k_setup_factor : stage bounds/penalties and the Riccati factor (role of
//                    Eq. (ldl), once per solve), written to the workspace as
//                    K_k, A_cl,k = A_k + B_k K_k, H_k^{-1} and s_k = P_{k+1} c_k.
//   k_admm         : all ADMM iterations (role of Eqs. (backsolve_1)-(backsolve_2)
//                    plus projection and dual update, Alg. 1's QP loop).
//   k_residual     : FP64 KKT residuals and objective of the returned iterate.
//   k_advance      : closed-loop plant step x0 <- A_0 x0 + B_0 u_0 + c_0 + noise.
//
// The back-sweep is run in closed-loop form: with g_k = qt_k + K_k' rt_k,
//   p'_k = p_{k+1} + s_k,  p_k = g_k + A_cl,k' p'_k,  d_k = -H_k^{-1}(rt_k + B_k' p'_k)
// and the rollout as x_{k+1} = A_cl,k x_k + (B_k d_k + c_k), u_k = K_k x_k + d_k,
// which is the textbook sweep (p_k = qt_k + A_k' p' + K_k' h, u_k = K_k x_k + d_k,
// x_{k+1} = A_k x_k + B_k u_k + c_k) with K_k' B_k' p' folded into A_cl,k'.  The
// serial chains then carry one nx x nx product per stage; everything else is
// independent across stages.
#include <math.h>

#include "factor_stage.h"
#include "generic_ops.h"
#include "mpc_internal.h"
#include "stage_rows.h"
#include "xlane.h"

#include <mutex>

namespace mpc {


template <typename T>
__global__ void __launch_bounds__(256)
k_setup_factor(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
               Inputs<T> in, SolverConsts sc_all, T* __restrict__ ws, int32_t* __restrict__ status) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, a);
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // The Riccati recursion runs in double for every io type T: inputs are
  // widened on load and the operators are rounded to T once when stored.
  // (Rounding P_k to float at every stage perturbs the operators by ~1e-6
  // relative, which 50 ADMM iterations amplify well past 1e-5.)
  using D = double;
  D* H = reinterpret_cast<D*>(smem_raw);   // H_k -> L_k               nu*nu
  D* P = H + nu * nu;                      // P_{k+1}, then P_k        nx*nx
  D* Ak = P + nx * nx;                     // A_k                      nx*nx
  D* PA = Ak + nx * nx;                    // P_{k+1} A_k              nx*nx
  D* Bk = PA + nx * nx;                    // B_k                      nx*nu
  D* PB = Bk + nx * nu;                    // P_{k+1} B_k, then K_k    nx*nu
  D* G = PB + nx * nu;                     // B_k' P A_k               nu*nx
  D* rdg = G + nu * nx;                    // diag Rt_k                nu
  D* rhok = rdg + nu;                      // row penalties of stage k m
  __shared__ int s_flag;

  const T* q = in.q + d.oq;
  const T* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  // workspace: K, A_cl, H^-1, s per stage (written by factor_stage), then the row bounds
  T* wl = ws + d.ows + (int64_t)N * (nu * nx + nx * nx + nu * nu + nx);
  T* wh = wl + (int64_t)N * m;
  T* wrho = wh + (int64_t)N * m;

  // Non-finite inputs mark the agent and stop it (no other agent is touched).
  if (tid == 0) s_flag = 0;
  __syncthreads();
  if (!agent_inputs_ok(in, d, tid, nt)) atomicOr(&s_flag, 1);
  __syncthreads();
  if (s_flag) {
    if (tid == 0) status[a] = AGENT_NONFINITE;
    return;
  }

  // Stage bounds and penalties (a1).
  for (int idx = tid; idx < N * m; idx += nt) {
    const int k = idx / m, i = idx % m;
    T lo, hi, rr;
    row_bounds<T, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rr);
    wl[idx] = lo;
    wh[idx] = hi;
    wrho[idx] = rr;
  }
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    P[idx] = ((i == j) ? (D)q[i] + sc.sigma + state_rho<D>(in, d, i, sc) : 0.0) +
             contact_weight<D>(in, d, N, i, j, sc);
  }
  __syncthreads();

  for (int k = N - 1; k >= 0; --k) {
    FactorLds<D> F{H, P, Ak, PA, Bk, PB, G, rdg, rhok};
    if (!factor_stage<T>(in, sc, d, k, F, ws, &s_flag, true, tid, nt)) {
      if (tid == 0) status[a] = AGENT_NOT_PD;
      return;
    }
  }
  if (tid == 0) status[a] = AGENT_OK;
}

// Rollout under the exact dynamics with gains K:  u_k = K_k x_k + d_k,
// x_{k+1} = A_k x_k + B_k u_k (+ c_k).  x_0 is x0p (zero if NULL); x_{k+1} is
// written to Xn[k]; u may alias d (each entry reads only its own d).
template <typename T, typename V>
__device__ inline void forward_exact(int N, int nx, int nu, const T* A, const T* B, const T* c,
                                     const T* wK, const V* d, const V* x0p, V* Xn, V* u, int tid,
                                     int nt) {
  const int qd = tid >> 2, sub = tid & 3, nq = nt >> 2;
  for (int k = 0; k < N; ++k) {
    const V* xk = k == 0 ? x0p : Xn + (k - 1) * nx;
    const T* Kk = wK + (int64_t)k * nu * nx;
    const T* Ak = A + (int64_t)k * nx * nx;
    const T* Bk = B + (int64_t)k * nx * nu;
    if (xk)
      quad_matvec<V>(nu, nx, [&](int j, int t) { return Kk[j * nx + t]; }, xk,
                     [&](int j, V acc) { u[k * nu + j] = d[k * nu + j] + acc; }, tid, nt);
    else
      for (int j = tid; j < nu; j += nt) u[k * nu + j] = d[k * nu + j];
    __syncthreads();
    const V* uk = u + k * nu;
    for (int i0 = 0; i0 < nx; i0 += nq) {
      const int i = i0 + qd;
      if (i < nx) {  // uniform within a quad
        V acc = 0;
        if (xk) acc = blocked_sum<V>(sub, 4, nx, [&](int t) { return (V)Ak[i * nx + t] * xk[t]; });
        acc += blocked_sum<V>(sub, 4, nu, [&](int t) { return (V)Bk[i * nu + t] * uk[t]; });
        acc = quad_sum(acc);
        if (sub == 0) Xn[k * nx + i] = c ? (V)c[(int64_t)k * nx + i] + acc : acc;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_admm(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
       Inputs<T> in, SolverConsts sc_all, int iters, int warm, const T* __restrict__ ws, State<T> st,
       int sweeps, double rtol) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, a);
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* X = st.x + d.ox;
  T* U = st.u + d.ou;
  T* Z = st.z + d.oz;
  T* Y = st.y + d.oy;
  if (st.status[a] != AGENT_OK) {
    const T nan = (T)NAN;
    for (int i = tid; i < (N + 1) * nx; i += nt) X[i] = nan;
    for (int i = tid; i < N * nu; i += nt) U[i] = nan;
    for (int i = tid; i < N * m; i += nt) {
      Z[i] = nan;
      Y[i] = nan;
    }
    if (st.zx)
      for (int i = tid; i < N * nx; i += nt) {
        st.zx[d.oc + i] = nan;
        st.yx[d.oc + i] = nan;
      }
    if (st.zc)
      for (int i = tid; i < N * d.n_feet * d.foot_dim; i += nt) {
        st.zc[d.ozc + i] = nan;
        st.yc[d.ozc + i] = nan;
      }
    return;
  }
  // Operators are read in the io type T; every vector, every accumulation and
  // the relaxation / projection / dual update run in double (on this chip the
  // FP64 VALU rate equals the non-packed FP32 rate).  Each product sum is
  // formed first and its offset added last, because offset and sum nearly
  // cancel (e.g. h = rt + B' p').
  using V = double;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* x = reinterpret_cast<V*>(smem_raw);  // (N+1)*nx
  V* xt = x + (N + 1) * nx;               // (N+1)*nx
  V* u = xt + (N + 1) * nx;               // N*nu
  V* ut = u + N * nu;                     // N*nu
  V* rt = ut + N * nu;                    // N*nu
  V* dv = rt + N * nu;                    // N*nu
  V* z = dv + N * nu;                     // N*m
  V* y = z + N * m;                       // N*m
  V* g = y + N * m;                       // N*nx
  V* pp = g + N * nx;                     // N*nx
  V* e = pp + N * nx;                     // N*nx
  V* p = e + N * nx;                      // nx
  V* hv = p + nx;                         // N*nu
  V* red = hv + N * nu;                   // 256 (refinement stopping test)
  // joint-limit rows (with limits): z_x, y_x of x_1..x_N
  const bool lim = in.xlo != nullptr;
  V* zx = red + 256;                      // N*nx
  V* yx = zx + N * nx;                    // N*nx
  // no-slip rows (with them): z_c, y_c of x_1..x_N and w_c = y_c - rho_c z_c
  const bool ctc = in.J != nullptr;
  const int nc = ctc ? d.n_feet * d.foot_dim : 0;
  V* zc = zx + (lim ? 2 * N * nx : 0);    // N*nc
  V* yc = zc + N * nc;                    // N*nc
  V* wc = yc + N * nc;                    // N*nc
  const T* Jc = ctc ? in.J + d.oJ : nullptr;

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
  const T* wK = ws + d.ows;
  const T* wAcl = wK + (int64_t)N * nu * nx;
  const T* wHi = wAcl + (int64_t)N * nx * nx;
  const T* wS = wHi + (int64_t)N * nu * nu;
  const T* wrho = wS + (int64_t)N * nx + 2 * (int64_t)N * m;
  const V sigma = sc.sigma, alpha = sc.alpha, oma = 1.0 - sc.alpha;
  const bool mixed = sweeps >= 0;

  const bool wm = agent_warm(warm, d);
  for (int i = tid; i < N * nu; i += nt) u[i] = wm ? (V)U[i] : 0.0;
  for (int i = tid; i < N * m; i += nt) {
    z[i] = wm ? (V)Z[i] : 0.0;
    y[i] = wm ? (V)Y[i] : 0.0;
  }
  if (lim)
    for (int i = tid; i < N * nx; i += nt) {
      zx[i] = wm ? (V)st.zx[d.oc + i] : 0.0;
      yx[i] = wm ? (V)st.yx[d.oc + i] : 0.0;
    }
  for (int i = tid; i < N * nc; i += nt) {
    zc[i] = wm ? (V)st.zc[d.ozc + i] : 0.0;
    yc[i] = wm ? (V)st.yc[d.ozc + i] : 0.0;
  }
  for (int i = tid; i < nx; i += nt) {
    x[i] = (V)x0[i];
    xt[i] = (V)x0[i];
  }
  __syncthreads();
  // x^0: rollout of the dynamics under u^0.
  for (int k = 0; k < N; ++k) {
    for (int i = tid; i < nx; i += nt) {
      V acc = 0;
      const T* Ar = A + (int64_t)k * nx * nx + i * nx;
      const T* Br = B + (int64_t)k * nx * nu + i * nu;
      for (int t = 0; t < nx; ++t) acc += (V)Ar[t] * x[k * nx + t];
      for (int t = 0; t < nu; ++t) acc += (V)Br[t] * u[k * nu + t];
      x[(k + 1) * nx + i] = (V)c[(int64_t)k * nx + i] + acc;
    }
    __syncthreads();
  }

  for (int it = 0; it < iters; ++it) {
    // rt_k = -sigma u_k - R ubar_k + C_k'(y_k - rho_k z_k)
    for (int idx = tid; idx < N * nu; idx += nt) {
      const int k = idx / nu, j = idx % nu;
      const V* yk = y + k * m;
      const V* zk = z + k * m;
      const uint8_t* stk = stance + k * d.n_feet;
      auto w = [&](int i) {
        V lo, hi, rr;
        row_bounds<V, T>(d, i, stk, tau, sc, lo, hi, rr);
        return yk[i] - rr * zk[i];
      };
      V v = w(j);
      if (j >= d.n_tau) {
        const int f = (j - d.n_tau) / d.foot_dim, cc = (j - d.n_tau) % d.foot_dim;
        const int b0 = nu + 4 * f;
        if (cc == 0) v += w(b0) - w(b0 + 1);
        if (cc == 1) v += w(b0 + 2) - w(b0 + 3);
        if (cc == 2) v -= mu * (w(b0) + w(b0 + 1) + w(b0 + 2) + w(b0 + 3));
      }
      V acc = -sigma * u[idx] + v;
      if (uref) acc -= (V)r[j] * (V)uref[idx];
      rt[idx] = acc;
    }
    // w_c = y_c - rho_c z_c of the no-slip rows of x_1..x_N
    for (int idx = tid; idx < N * nc; idx += nt) {
      double rr;
      contact_row(d, stance, idx / nc + 1, idx % nc, sc, rr);
      wc[idx] = yc[idx] - (V)rr * zc[idx];
    }
    __syncthreads();
    // g_k = qt_k + K_k' rt_k, qt_k = -Q r_k - sigma x_k
    quad_dot<V>(N * nx, nu,
                [&](int idx, int j) {
                  const int k = idx / nx, i = idx % nx;
                  return (V)wK[((int64_t)k * nu + j) * nx + i] * rt[k * nu + j];
                },
                [&](int idx, V acc) {
                  const int k = idx / nx, i = idx % nx;
                  V qt = -(V)q[i] * (V)xr[(int64_t)k * nx + i] - sigma * x[idx];
                  if (lim && k >= 1)  // the state rows of x_k: y_x - rho_x z_x
                    qt += yx[idx - nx] - state_rho<V>(in, d, i, sc) * zx[idx - nx];
                  if (k >= 1)  // the no-slip rows of x_k: Jc' w_c,k
                    for (int row = 0; row < nc; ++row) qt += (V)Jc[row * nx + i] * wc[(k - 1) * nc + row];
                  g[idx] = qt + acc;
                },
                tid, nt);
    for (int i = tid; i < nx; i += nt) {
      V qt = -(V)q[i] * (V)xr[(int64_t)N * nx + i] - sigma * x[N * nx + i];
      if (lim) qt += yx[(N - 1) * nx + i] - state_rho<V>(in, d, i, sc) * zx[(N - 1) * nx + i];
      for (int row = 0; row < nc; ++row) qt += (V)Jc[row * nx + i] * wc[(N - 1) * nc + row];
      p[i] = qt;
    }
    __syncthreads();
    // backward chain: p'_k = p_{k+1} + s_k, p_k = g_k + A_cl,k' p'_k
    for (int k = N - 1; k >= 0; --k) {
      for (int i = tid; i < nx; i += nt) pp[k * nx + i] = p[i] + (V)wS[(int64_t)k * nx + i];
      __syncthreads();
      if (k > 0) {
        const T* Ac = wAcl + (int64_t)k * nx * nx;
        quad_matvec<V>(nx, nx, [&](int i, int t) { return Ac[t * nx + i]; }, pp + k * nx,
                       [&](int i, V acc) { p[i] = g[k * nx + i] + acc; }, tid, nt);
        __syncthreads();
      }
    }
    // d_k = -H_k^{-1}(rt_k + B_k' p'_k),  e_k = B_k d_k + c_k
    quad_dot<V>(N * nu, nx,
                [&](int idx, int t) {
                  const int k = idx / nu, j = idx % nu;
                  return (V)B[((int64_t)k * nx + t) * nu + j] * pp[k * nx + t];
                },
                [&](int idx, V acc) { hv[idx] = rt[idx] + acc; }, tid, nt);
    __syncthreads();
    quad_dot<V>(N * nu, nu,
                [&](int idx, int t) {
                  const int k = idx / nu, j = idx % nu;
                  return (V)wHi[((int64_t)k * nu + j) * nu + t] * hv[k * nu + t];
                },
                [&](int idx, V acc) { dv[idx] = -acc; }, tid, nt);
    __syncthreads();
    if (!mixed) {
      quad_dot<V>(N * nx, nu,
                  [&](int idx, int t) {
                    const int k = idx / nx;
                    return (V)B[(int64_t)idx * nu + t] * dv[k * nu + t];
                  },
                  [&](int idx, V acc) { e[idx] = (V)c[idx] + acc; }, tid, nt);
      __syncthreads();
      // forward chain: xt_{k+1} = A_cl,k xt_k + e_k
      for (int k = 0; k < N; ++k) {
        const T* Ak = wAcl + (int64_t)k * nx * nx;
        quad_matvec<V>(nx, nx, [&](int i, int t) { return Ak[i * nx + t]; }, xt + k * nx,
                       [&](int i, V acc) { xt[(k + 1) * nx + i] = e[k * nx + i] + acc; }, tid, nt);
        __syncthreads();
      }
      // ut_k = K_k xt_k + d_k
      quad_dot<V>(N * nu, nx,
                  [&](int idx, int t) {
                    const int k = idx / nu;
                    return (V)wK[(int64_t)idx * nx + t] * xt[k * nx + t];
                  },
                  [&](int idx, V acc) { ut[idx] = dv[idx] + acc; }, tid, nt);
      __syncthreads();
    } else {
      // Mixed precision: the gains come from low-precision products, so the
      // rollout runs under the exact dynamics (ut_k = K_k xt_k + d_k,
      // xt_{k+1} = A_k xt_k + B_k ut_k + c_k) and only the stationarity of
      // the x-subproblem is left to refine.
      forward_exact<T, V>(N, nx, nu, A, B, c, wK, dv, xt, xt + nx, ut, tid, nt);
      // b = (qt, rt): scale of the stopping test
      V bl = 0;
      for (int idx = nx + tid; idx < (N + 1) * nx; idx += nt) {
        const int i = idx % nx;
        bl = fmax(bl, fabs(-(V)q[i] * (V)xr[idx] - sigma * x[idx]));
      }
      for (int idx = tid; idx < N * nu; idx += nt) bl = fmax(bl, fabs(rt[idx]));
      const V bn = block_max(bl, red);
      for (int sw = 0; sw < sweeps; ++sw) {
        // costates of the x-subproblem at (xt, ut) from its x-stationarity:
        // lam_N = Qt xt_N + qt_N, lam_k = Qt xt_k + qt_k + A_k' lam_{k+1};
        // lam_{k+1} is kept in pp[k]
        for (int i = tid; i < nx; i += nt) {
          const int idx = N * nx + i;
          pp[(N - 1) * nx + i] = ((V)q[i] + sigma) * xt[idx] + (-(V)q[i] * (V)xr[idx] - sigma * x[idx]);
        }
        __syncthreads();
        for (int k = N - 1; k >= 1; --k) {
          const T* Ac = A + (int64_t)k * nx * nx;
          quad_matvec<V>(nx, nx, [&](int i, int t) { return Ac[t * nx + i]; }, pp + k * nx,
                         [&](int i, V acc) {
                           const int idx = k * nx + i;
                           pp[(k - 1) * nx + i] = ((V)q[i] + sigma) * xt[idx] +
                                                  (-(V)q[i] * (V)xr[idx] - sigma * x[idx]) + acc;
                         },
                         tid, nt);
          __syncthreads();
        }
        // u-stationarity residual ru_k = Rt_k ut_k + rt_k + B_k' lam_{k+1}
        V rl = 0;
        for (int idx = tid; idx < N * nu; idx += nt) {
          const int k = idx / nu, j = idx % nu;
          const T* Bc = B + (int64_t)k * nx * nu + j;
          const V acc = blocked_sum<V>(0, 1, nx, [&](int t) { return (V)Bc[t * nu] * pp[k * nx + t]; });
          const V rtd = rtilde_diag<V, T>(d, j, (V)r[j], mu, wrho + (int64_t)k * m, sc);
          hv[idx] = rtd * ut[idx] + rt[idx] + acc;
          rl = fmax(rl, fabs(hv[idx]));
        }
        const V rn = block_max(rl, red);
        if (!(rn > rtol * bn)) break;
        // correction: the same LQR with linear term ru, no offsets, x_0 fixed,
        // solved with the low-precision factor
        for (int idx = tid; idx < N * nx; idx += nt) {
          const int k = idx / nx, i = idx % nx;
          const T* Kc = wK + (int64_t)k * nu * nx + i;
          g[idx] = blocked_sum<V>(0, 1, nu, [&](int j) { return (V)Kc[j * nx] * hv[k * nu + j]; });
        }
        for (int i = tid; i < nx; i += nt) p[i] = 0;
        __syncthreads();
        for (int k = N - 1; k >= 0; --k) {
          for (int i = tid; i < nx; i += nt) e[k * nx + i] = p[i];
          __syncthreads();
          if (k > 0) {
            const T* Ac = wAcl + (int64_t)k * nx * nx;
            quad_matvec<V>(nx, nx, [&](int i, int t) { return Ac[t * nx + i]; }, e + k * nx,
                           [&](int i, V acc) { p[i] = g[k * nx + i] + acc; }, tid, nt);
            __syncthreads();
          }
        }
        for (int idx = tid; idx < N * nu; idx += nt) {
          const int k = idx / nu, j = idx % nu;
          const T* Bc = B + (int64_t)k * nx * nu + j;
          hv[idx] = hv[idx] + blocked_sum<V>(0, 1, nx, [&](int t) { return (V)Bc[t * nu] * e[k * nx + t]; });
        }
        __syncthreads();
        for (int idx = tid; idx < N * nu; idx += nt) {
          const int k = idx / nu, j = idx % nu;
          const T* Hr = wHi + (int64_t)k * nu * nu + j * nu;
          dv[idx] = -blocked_sum<V>(0, 1, nu, [&](int t) { return (V)Hr[t] * hv[k * nu + t]; });
        }
        __syncthreads();
        // dx (in g, dx_{k+1} at g[k]) and du (in dv) under the exact dynamics
        forward_exact<T, V>(N, nx, nu, A, B, (const T*)nullptr, wK, dv, (const V*)nullptr, g, dv,
                            tid, nt);
        for (int idx = nx + tid; idx < (N + 1) * nx; idx += nt) xt[idx] += g[idx - nx];
        for (int idx = tid; idx < N * nu; idx += nt) ut[idx] += dv[idx];
        __syncthreads();
      }
    }
    // relaxation, projection onto [l, h], dual update (the joint-limit rows
    // take xt_k, k = 1..N, before x is relaxed)
    if (lim)
      for (int idx = tid; idx < N * nx; idx += nt) {
        const int i = idx % nx;
        const V rr = state_rho<V>(in, d, i, sc);
        const V lo = (V)in.xlo[d.oq + i], hi = (V)in.xhi[d.oq + i];
        const V w = alpha * xt[idx + nx] + oma * zx[idx];
        const V zn = fmin(fmax(w + yx[idx] / rr, lo), hi);
        yx[idx] = yx[idx] + rr * (w - zn);
        zx[idx] = zn;
      }
    // the no-slip rows take Jc xt_k (k = 1..N): equality rows project to 0,
    // free rows keep w + y_c / rho_c
    if (ctc)
      quad_dot<V>(N * nc, nx,
                  [&](int idx, int t) { return (V)Jc[(idx % nc) * nx + t] * xt[(idx / nc + 1) * nx + t]; },
                  [&](int idx, V zeta) {
                    double rr;
                    const bool eq = contact_row(d, stance, idx / nc + 1, idx % nc, sc, rr);
                    const V w = alpha * zeta + oma * zc[idx];
                    const V zn = eq ? (V)0 : w + yc[idx] / (V)rr;
                    yc[idx] = yc[idx] + (V)rr * (w - zn);
                    zc[idx] = zn;
                  },
                  tid, nt);
    for (int idx = nx + tid; idx < (N + 1) * nx; idx += nt) x[idx] = alpha * xt[idx] + oma * x[idx];
    for (int idx = tid; idx < N * m; idx += nt) {
      const int k = idx / m, i = idx % m;
      V lo, hi, rr;
      row_bounds<V, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rr);
      const V zeta = c_row<V>(d, i, mu, ut + k * nu);
      const V w = alpha * zeta + oma * z[idx];
      const V zn = fmin(fmax(w + y[idx] / rr, lo), hi);
      y[idx] = y[idx] + rr * (w - zn);
      z[idx] = zn;
    }
    __syncthreads();
    for (int idx = tid; idx < N * nu; idx += nt) u[idx] = alpha * ut[idx] + oma * u[idx];
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
  if (lim)
    for (int i = tid; i < N * nx; i += nt) {
      st.zx[d.oc + i] = (T)zx[i];
      st.yx[d.oc + i] = (T)yx[i];
      ok &= (bool)isfinite(zx[i]) && (bool)isfinite(yx[i]);
    }
  for (int i = tid; i < N * nc; i += nt) {
    st.zc[d.ozc + i] = (T)zc[i];
    st.yc[d.ozc + i] = (T)yc[i];
    ok &= (bool)isfinite(zc[i]) && (bool)isfinite(yc[i]);
  }
  if (!ok) st.status[a] = AGENT_NONFINITE;
}

// Workgroup max of rp, rd, ry, rc and sum of obj, valid in thread 0: a
// butterfly within each wavefront, then one exchange of the wavefronts' values.
__device__ inline void block_reduce_res(double& rp, double& rd, double& ry, double& rc, double& obj,
                                        double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    rp = fmax(rp, __shfl_xor(rp, off));
    rd = fmax(rd, __shfl_xor(rd, off));
    ry = fmax(ry, __shfl_xor(ry, off));
    rc = fmax(rc, __shfl_xor(rc, off));
    obj += __shfl_xor(obj, off);
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[5 * w] = rp;
    red[5 * w + 1] = rd;
    red[5 * w + 2] = ry;
    red[5 * w + 3] = rc;
    red[5 * w + 4] = obj;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int v = 1; v < nw; ++v) {
      rp = fmax(rp, red[5 * v]);
      rd = fmax(rd, red[5 * v + 1]);
      ry = fmax(ry, red[5 * v + 2]);
      rc = fmax(rc, red[5 * v + 3]);
      obj += red[5 * v + 4];
    }
}

// FP64 KKT residuals of the returned iterate (the role of the solution check
// that follows the QP loop in Alg. 1).  Costates of the dynamics rows come from
// the adjoint sweep lambda_N = Q(x_N - r_N), lambda_k = Q(x_k - r_k) + A_k' lambda_{k+1}.
template <typename T>
__global__ void __launch_bounds__(256)
k_residual(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
           Inputs<T> in, SolverConsts sc_all, State<T> st) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, a);
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;  // nt = 256
  // every dot product is split over the 4 lanes of a quad (terms t = sub,
  // sub + 4, ...) and summed with DPP; quad qd owns output qd (nx <= 64)
  const int qd = tid >> 2, sub = tid & 3;
  __shared__ double red[256];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lam = reinterpret_cast<double*>(smem_raw);     // (N+1)*nx
  if (st.status[a] != AGENT_OK && st.status[a] != AGENT_CONVERGED) {
    if (tid < 4) st.res[(int64_t)a * 4 + tid] = NAN;
    if (tid == 0) st.obj[a] = (T)NAN;
    return;
  }
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
  const double mu = (double)in.mu[d.omu];
  const T* x = st.x + d.ox;
  const T* u = st.u + d.ou;
  const T* z = st.z + d.oz;
  const T* y = st.y + d.oy;

  double* xs = lam + (N + 1) * nx;                      // x as double  (N+1)*nx
  double* us = xs + (N + 1) * nx;                       // u as double  N*nu
  T* As = reinterpret_cast<T*>(us + N * nu);            // nx x (nx+1)
  T* Bs = As + nx * (nx + 1);                           // nx x (nu+1)

  // Stage by stage, k = N-1 .. 0, every residual that involves A_k and B_k is
  // formed from LDS: lambda_k = Q(x_k - r_k) + A_k' lambda_{k+1}, the dual
  // residual of u_k, R(u_k - ubar_k) + B_k' lambda_{k+1} + C_k' y_k, and the
  // dynamics residual x_{k+1} - A_k x_k - B_k u_k - c_k.  Stage k-1's A, B and
  // the per-output terms that come from HBM are loaded into registers while
  // stage k is computed (a quad owns output qd of each product).
  constexpr int kPA = (64 * 64 + 255) / 256, kPB = (64 * 32 + 255) / 256;
  T ra[kPA], rb[kPB];
  double cdyn = 0.0, cdual = 0.0;
  const float inx = 1.0f / (float)nx, inu = 1.0f / (float)nu;
  auto fetch = [&](int k) {
    const T* Ag = A + (int64_t)k * nx * nx;
    const T* Bg = B + (int64_t)k * nx * nu;
#pragma unroll
    for (int t = 0; t < kPA; ++t) {
      const int e = tid + t * nt;
      ra[t] = e < nx * nx ? Ag[e] : (T)0;
    }
#pragma unroll
    for (int t = 0; t < kPB; ++t) {
      const int e = tid + t * nt;
      rb[t] = e < nx * nu ? Bg[e] : (T)0;
    }
    // x_{k+1} - c_k of output qd, and R(u_k - ubar_k) + C_k' y_k of input qd
    if (qd < nx) cdyn = (double)x[(k + 1) * nx + qd] - (double)c[(int64_t)k * nx + qd];
    if (qd < nu) {
      const int o = k * nu + qd;
      double v = (double)r[qd] * ((double)u[o] - (uref ? (double)uref[o] : 0.0));
      const T* yk = y + k * m;
      v += (double)yk[qd];
      if (qd >= d.n_tau) {
        const int f = (qd - d.n_tau) / d.foot_dim, cc = (qd - d.n_tau) % d.foot_dim;
        const T* yp = yk + nu + 4 * f;
        if (cc == 0) v += (double)yp[0] - (double)yp[1];
        if (cc == 1) v += (double)yp[2] - (double)yp[3];
        if (cc == 2) v -= mu * ((double)yp[0] + (double)yp[1] + (double)yp[2] + (double)yp[3]);
      }
      cdual = v;
    }
  };
  fetch(N - 1);  // first: its loads overlap the element-wise pass below
  // One pass over the element-wise terms, its loads issued together: x and u
  // into LDS as double, lambda_k = Q(x_k - r_k) (A_k' lambda_{k+1} is added
  // stage by stage), the objective, x_0's residual, and the row residuals
  // (primal C u - z and complementarity of y with the bounds)
  double obj = 0.0, rp = 0.0, rd = 0.0, ry = 0.0, rc = 0.0;
  {
    const int nX = (N + 1) * nx, nU = N * nu, nR = N * m;
    const int nmax = nX > nU ? (nX > nR ? nX : nR) : (nU > nR ? nU : nR);
    for (int idx = tid; idx < nmax; idx += nt) {
      if (idx < nX) {
        const double xv = (double)x[idx];
        xs[idx] = xv;
        const double ee = xv - (double)xr[idx];
        lam[idx] = (double)q[idx % nx] * ee;
        if (idx >= nx) obj += 0.5 * (double)q[idx % nx] * ee * ee;
        else ry = fmax(ry, fabs(xv - (double)x0[idx]));
        if (in.xlo && idx >= nx) {  // joint-limit row of x_k: multiplier, primal, complementarity
          const int i = idx % nx;
          const double zz = (double)st.zx[d.oc + idx - nx], yy = (double)st.yx[d.oc + idx - nx];
          lam[idx] += yy;
          rp = fmax(rp, fabs(xv - zz));
          const double lo = (double)in.xlo[d.oq + i], hi = (double)in.xhi[d.oq + i];
          const double yp = yy > 0.0 ? yy : 0.0, ym = yy < 0.0 ? -yy : 0.0;
          const double ca = isinf(hi) ? yp : fmin(yp, hi - zz);
          const double cb = isinf(lo) ? ym : fmin(ym, zz - lo);
          rc = fmax(rc, fmax(fabs(ca), fabs(cb)));
          if (zz > hi) rc = fmax(rc, zz - hi);
          if (zz < lo) rc = fmax(rc, lo - zz);
        }
        if (in.J && idx >= nx) {  // no-slip rows of x_k: Jc' y_c,k joins the costate
          const int i = idx % nx, k = idx / nx, ncr = d.n_feet * d.foot_dim;
          const T* Jc = in.J + d.oJ;
          const T* yck = st.yc + d.ozc + (int64_t)(k - 1) * ncr;
          double acc = 0.0;
          for (int row = 0; row < ncr; ++row) acc += (double)Jc[row * nx + i] * (double)yck[row];
          lam[idx] += acc;
        }
      }
      if (idx < nU) {
        const double uv = (double)u[idx];
        us[idx] = uv;
        const double ee = uv - (uref ? (double)uref[idx] : 0.0);
        obj += 0.5 * (double)r[idx % nu] * ee * ee;
      }
      if (idx < nR) {
        const int k = idx / m, i = idx % m;
        double cu;
        const T* uk = u + k * nu;
        if (i < nu) {
          cu = (double)uk[i];
        } else {
          const int f = (i - nu) >> 2, pp = (i - nu) & 3, b = d.n_tau + f * d.foot_dim;
          const double t = (pp < 2) ? (double)uk[b] : (double)uk[b + 1];
          cu = ((pp & 1) ? -t : t) - mu * (double)uk[b + 2];
        }
        rp = fmax(rp, fabs(cu - (double)z[idx]));
        T lo_t, hi_t, rho_t;
        row_bounds<T, T>(d, i, stance + k * d.n_feet, tau, sc, lo_t, hi_t, rho_t);
        const double lo = (double)lo_t, hi = (double)hi_t, zz = (double)z[idx], yy = (double)y[idx];
        const double yp = yy > 0.0 ? yy : 0.0, ym = yy < 0.0 ? -yy : 0.0;
        const double ca = isinf(hi) ? yp : fmin(yp, hi - zz);
        const double cb = isinf(lo) ? ym : fmin(ym, zz - lo);
        rc = fmax(rc, fmax(fabs(ca), fabs(cb)));
        if (zz > hi) rc = fmax(rc, zz - hi);
        if (zz < lo) rc = fmax(rc, lo - zz);
      }
    }
    // no-slip rows of x_1..x_N: primal |Jc x_k - z_c| and complementarity
    // (equality rows: z_c = 0; free rows: y_c = 0)
    if (in.J) {
      const int ncr = d.n_feet * d.foot_dim;
      const T* Jc = in.J + d.oJ;
      for (int idx = tid; idx < N * ncr; idx += nt) {
        const int k = idx / ncr + 1, row = idx % ncr;
        double jx = 0.0;
        for (int t = 0; t < nx; ++t) jx += (double)Jc[row * nx + t] * (double)x[k * nx + t];
        const double zz = (double)st.zc[d.ozc + idx], yy = (double)st.yc[d.ozc + idx];
        rp = fmax(rp, fabs(jx - zz));
        double rr;
        if (contact_row(d, stance, k, row, sc, rr))
          rc = fmax(rc, fabs(zz));
        else
          rc = fmax(rc, fabs(yy));
      }
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    __syncthreads();  // the previous stage's readers of As, Bs and lambda are done
    // rows padded by one element (row = e / n through a float reciprocal:
    // exact here, the fraction (e mod n + 1/2) / n stays 1/(2n) away from 0 and 1)
#pragma unroll
    for (int t = 0; t < kPA; ++t) {
      const int e = tid + t * nt;
      if (e < nx * nx) {
        const int row = (int)(((float)e + 0.5f) * inx);
        As[row * (nx + 1) + (e - row * nx)] = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < kPB; ++t) {
      const int e = tid + t * nt;
      if (e < nx * nu) {
        const int row = (int)(((float)e + 0.5f) * inu);
        Bs[row * (nu + 1) + (e - row * nu)] = rb[t];
      }
    }
    const double cd = cdyn, cu = cdual;
    __syncthreads();
    if (k >= 1) fetch(k - 1);
    const double* lk1 = lam + (k + 1) * nx;
    if (k >= 1 && qd < nx) {
      double acc = 0.0;
      for (int t = sub; t < nx; t += 4) acc += (double)As[t * (nx + 1) + qd] * lk1[t];
      acc = quad_sum(acc);
      if (sub == 0) lam[k * nx + qd] += acc;
    }
    if (qd < nu) {
      double acc = 0.0;
      for (int t = sub; t < nx; t += 4) acc += (double)Bs[t * (nu + 1) + qd] * lk1[t];
      acc = quad_sum(acc);
      if (sub == 0) rd = fmax(rd, fabs(acc + cu));
    }
    if (qd < nx) {
      double acc = 0.0;
      const double* xk = xs + k * nx;
      const double* uk = us + k * nu;
      for (int t = sub; t < nx; t += 4) acc += (double)As[qd * (nx + 1) + t] * xk[t];
      for (int t = sub; t < nu; t += 4) acc += (double)Bs[qd * (nu + 1) + t] * uk[t];
      acc = quad_sum(acc);
      if (sub == 0) ry = fmax(ry, fabs(cd - acc));
    }
  }
  __syncthreads();
  block_reduce_res(rp, rd, ry, rc, obj, red);
  if (tid == 0) {
    double* res = st.res + (int64_t)a * 4;
    res[0] = rp;
    res[1] = rd;
    res[2] = ry;
    res[3] = rc;
    st.obj[a] = (T)obj;
  }
}

template <typename T>
__global__ void __launch_bounds__(64)
k_advance(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
          Inputs<T> in, const T* __restrict__ u, const T* __restrict__ noise, T* __restrict__ x0n) {
  if ((int)blockIdx.x >= n_launch) return;
  const int a = list ? list[blockIdx.x] : (int)blockIdx.x;
  const AgentDesc d = desc[a];
  const int nx = d.nx, nu = d.nu;
  const T* A0 = in.A + d.oA;
  const T* B0 = in.B + d.oB;
  const T* x0 = in.x0 + d.ox0;
  const T* u0 = u + d.ou;
  T acc[2] = {0, 0};
  for (int r = 0; r < 2; ++r) {
    const int i = threadIdx.x + r * 64;
    if (i < nx) {
      T v = in.c[d.oc + i] + (noise ? noise[d.ox0 + i] : (T)0);
      for (int t = 0; t < nx; ++t) v += A0[i * nx + t] * x0[t];
      for (int t = 0; t < nu; ++t) v += B0[i * nu + t] * u0[t];
      acc[r] = v;
    }
  }
  __syncthreads();  // x0n may alias x0: all reads finish before any write
  for (int r = 0; r < 2; ++r) {
    const int i = threadIdx.x + r * 64;
    if (i < nx) x0n[d.ox0 + i] = acc[r];
  }
}

template <typename T>
hipError_t launch_generic_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch,
                                 Inputs<T> in, SolverConsts sc, T* ws, int32_t* status, size_t lds,
                                 int threads, hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_setup_factor<T>, dim3(n_launch), dim3(threads), lds, stream, d_desc, list,
                     n_launch, in, sc, ws, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_generic_admm(const AgentDesc* d_desc, const int32_t* list, int n_launch,
                               Inputs<T> in, SolverConsts sc, int iters, int warm, const T* ws,
                               State<T> st, size_t lds, int threads, hipStream_t stream,
                               int sweeps, double rtol) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_admm<T>, dim3(n_launch), dim3(threads), lds, stream, d_desc, list, n_launch,
                     in, sc, iters, warm, ws, st, sweeps, rtol);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                           SolverConsts sc, State<T> st, size_t lds, hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual<T>, dim3(n_launch), dim3(256), lds, stream, d_desc, list,
                     n_launch, in, sc, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_advance(const AgentDesc* d_desc, const int32_t* list, int n_launch, Inputs<T> in,
                          const T* u, const T* noise, T* x0_next, hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_advance<T>, dim3(n_launch), dim3(64), 0, stream, d_desc, list, n_launch,
                     in, u, noise, x0_next);
  return hipGetLastError();
}

// The limits are per kernel and process-wide (every plan and server shares
// them), so they only ever grow: a limit has no effect on occupancy, and
// lowering it would break launches of an earlier plan.
hipError_t generic_set_lds_limits(size_t lds_factor, size_t lds_admm, size_t lds_res) {
  static std::mutex mu;
  static size_t cur[3] = {0, 0, 0};
  std::lock_guard<std::mutex> lock(mu);
  hipError_t e = hipSuccess;
#define MPC_SET(kern, bytes)                                                                  \
  if (e == hipSuccess)                                                                        \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes));
  if (lds_factor > cur[0]) {
    MPC_SET(k_setup_factor<float>, lds_factor)
    MPC_SET(k_setup_factor<double>, lds_factor)
    if (e == hipSuccess) cur[0] = lds_factor;
  }
  if (lds_admm > cur[1]) {
    MPC_SET(k_admm<float>, lds_admm)
    MPC_SET(k_admm<double>, lds_admm)
    if (e == hipSuccess) cur[1] = lds_admm;
  }
  if (lds_res > cur[2]) {
    MPC_SET(k_residual<float>, lds_res)
    MPC_SET(k_residual<double>, lds_res)
    if (e == hipSuccess) cur[2] = lds_res;
  }
#undef MPC_SET
  return e;
}

#define MPC_INSTANTIATE(T)                                                                        \
  template hipError_t launch_generic_factor<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,  \
                                               SolverConsts, T*, int32_t*, size_t, int,           \
                                               hipStream_t);                                      \
  template hipError_t launch_generic_admm<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,    \
                                             SolverConsts, int, int, const T*, State<T>, size_t,  \
                                             int, hipStream_t, int, double);                      \
  template hipError_t launch_residual<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,        \
                                         SolverConsts, State<T>, size_t, hipStream_t);            \
  template hipError_t launch_advance<T>(const AgentDesc*, const int32_t*, int, Inputs<T>,         \
                                        const T*, const T*, T*, hipStream_t);
MPC_INSTANTIATE(float)
MPC_INSTANTIATE(double)

}  // namespace mpc
