// One stage of the Riccati factor (role of Eq. (ldl)) from P_{k+1}: the stage's
// penalties, H_k = Rt_k + B_k' P B_k (Cholesky, FP64), G_k = B_k' P A_k,
// K_k = -H_k^{-1} G_k, A_cl,k = A_k + B_k K_k, H_k^{-1} and s_k = P_{k+1} c_k
// written to the workspace; with update_P, P is then overwritten by
// P_k = Qt_k + A_k' P A_k + G_k' K_k (symmetrised).  Shared by the serial
// factor (stages N-1..0 in one workgroup) and the parallel-in-time factor
// (each stage in its own workgroup, P_{k+1} from the scan).  Returns false if
// H_k is not positive definite.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "generic_ops.h"
#include "mpc_internal.h"
#include "stage_rows.h"

namespace mpc {

// This thread's share of the check that an agent's inputs are finite (and its
// joint-limit intervals not empty); the workgroup combines the threads' results.
template <typename T>
__device__ inline bool agent_inputs_ok(const Inputs<T>& in, const AgentDesc& d, int tid, int nt) {
  const int N = d.N, nx = d.nx, nu = d.nu;
  bool ok = finite_all(in.A + d.oA, (int64_t)N * nx * nx, tid, nt) &&
            finite_all(in.B + d.oB, (int64_t)N * nx * nu, tid, nt) &&
            finite_all(in.c + d.oc, (int64_t)N * nx, tid, nt) && finite_all(in.q + d.oq, nx, tid, nt) &&
            finite_all(in.r + d.orr, nu, tid, nt) &&
            finite_all(in.xr + d.oxr, (int64_t)(N + 1) * nx, tid, nt) &&
            finite_all(in.x0 + d.ox0, nx, tid, nt) && finite_all(in.tau + d.otau, d.n_tau, tid, nt) &&
            (bool)isfinite(in.mu[d.omu]) &&
            (!in.uref || finite_all(in.uref + d.our, (int64_t)N * nu, tid, nt));
  if (in.xlo)
    for (int i = tid; i < nx; i += nt) {
      const T lo = in.xlo[d.oq + i], hi = in.xhi[d.oq + i];
      ok &= !isnan(lo) && !isnan(hi) && lo <= hi;
    }
  if (in.J) ok &= finite_all(in.J + d.oJ, (int64_t)d.n_feet * d.foot_dim * nx, tid, nt);
  return ok;
}

template <typename D>
struct FactorLds {
  D* H;     // H_k -> L_k               nu*nu
  D* P;     // P_{k+1}, then P_k        nx*nx
  D* Ak;    // A_k                      nx*nx
  D* PA;    // P_{k+1} A_k              nx*nx
  D* Bk;    // B_k                      nx*nu
  D* PB;    // P_{k+1} B_k, then K_k    nx*nu
  D* G;     // B_k' P A_k               nu*nx
  D* rdg;   // diag Rt_k                nu
  D* rhok;  // row penalties of stage k m
};

template <typename T>
__device__ inline bool factor_stage(const Inputs<T>& in, const SolverConsts& sc, const AgentDesc& d, int k,
                                    const FactorLds<double>& F, T* __restrict__ ws, int* s_flag,
                                    bool update_P, int tid, int nt) {
  using D = double;
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  D* H = F.H;
  D* P = F.P;
  D* Ak = F.Ak;
  D* PA = F.PA;
  D* Bk = F.Bk;
  D* PB = F.PB;
  D* Kk = F.PB;
  D* G = F.G;
  D* rdg = F.rdg;
  D* rhok = F.rhok;
  const T* A = in.A + d.oA;
  const T* B = in.B + d.oB;
  const T* c = in.c + d.oc;
  const T* q = in.q + d.oq;
  const T* r = in.r + d.orr;
  const T* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const T mu = in.mu[d.omu];
  T* wK = ws + d.ows;
  T* wAcl = wK + (int64_t)N * nu * nx;
  T* wHi = wAcl + (int64_t)N * nx * nx;
  T* wS = wHi + (int64_t)N * nu * nu;
  const T* Ag = A + (int64_t)k * nx * nx;
  const T* Bg = B + (int64_t)k * nx * nu;
  for (int idx = tid; idx < nx * nx; idx += nt) Ak[idx] = (D)Ag[idx];
  for (int idx = tid; idx < nx * nu; idx += nt) Bk[idx] = (D)Bg[idx];
  for (int i = tid; i < m; i += nt) {
    D lo, hi;
    row_bounds<D, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rhok[i]);
  }
  __syncthreads();
  for (int j = tid; j < nu; j += nt) rdg[j] = rtilde_diag<D, D>(d, j, (D)r[j], (D)mu, rhok, sc);
  __syncthreads();
  for (int idx = tid; idx < nx * nu; idx += nt) {
    const int i = idx / nu, j = idx % nu;
    PB[idx] = blocked_sum<D>(0, 1, nx, [&](int t) { return P[i * nx + t] * Bk[t * nu + j]; });
  }
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    PA[idx] = blocked_sum<D>(0, 1, nx, [&](int t) { return P[i * nx + t] * Ak[t * nx + j]; });
  }
  for (int i = tid; i < nx; i += nt) {
    const D acc = blocked_sum<D>(0, 1, nx, [&](int t) { return P[i * nx + t] * (D)c[(int64_t)k * nx + t]; });
    wS[(int64_t)k * nx + i] = (T)acc;
  }
  __syncthreads();
  for (int idx = tid; idx < nu * nu; idx += nt) {
    const int i = idx / nu, j = idx % nu;
    H[idx] = blocked_sum<D>(0, 1, nx, [&](int t) { return Bk[t * nu + i] * PB[t * nu + j]; },
                            (i == j) ? rdg[i] : 0.0);
  }
  for (int idx = tid; idx < nu * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    G[idx] = blocked_sum<D>(0, 1, nx, [&](int t) { return Bk[t * nu + i] * PA[t * nx + j]; });
  }
  __syncthreads();
  // Right-looking Cholesky of H_k in place (lower triangle).
  for (int j = 0; j < nu; ++j) {
    if (tid == 0) {
      const double v = H[j * nu + j];
      if (!(v > 0.0)) *s_flag = 1;
      H[j * nu + j] = sqrt(v);
    }
    __syncthreads();
    if (*s_flag) break;
    for (int i = j + 1 + tid; i < nu; i += nt) H[i * nu + j] /= H[j * nu + j];
    __syncthreads();
    const int rem = nu - j - 1;
    for (int idx = tid; idx < rem * rem; idx += nt) {
      const int i = j + 1 + idx / rem, cc = j + 1 + idx % rem;
      if (cc <= i) H[i * nu + cc] -= H[i * nu + j] * H[cc * nu + j];
    }
    __syncthreads();
  }
  if (*s_flag) return false;
  // K_k = -H_k^{-1} G_k into LDS (over the dead P B_k) and H_k^{-1} straight
  // into the workspace, one column per thread.
  // The column is carried in double registers (nu <= 32, loops unrolled so
  // the array stays in VGPRs) and rounded to T once at the end.
  for (int col = tid; col < nx + nu; col += nt) {
    const bool isK = col < nx;
    const int cc = isK ? col : col - nx;
    const int ld = isK ? nx : nu;
    double v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      if (i < nu) {
        double acc = isK ? -G[i * nx + cc] : (i == cc ? 1.0 : 0.0);
#pragma unroll
        for (int t = 0; t < i; ++t) acc -= H[i * nu + t] * v[t];
        v[i] = acc / H[i * nu + i];
      }
    }
#pragma unroll
    for (int i = 31; i >= 0; --i) {
      if (i < nu) {
        double acc = v[i];
#pragma unroll
        for (int t = i + 1; t < 32; ++t)
          if (t < nu) acc -= H[t * nu + i] * v[t];
        v[i] = acc / H[i * nu + i];
      }
    }
    if (isK) {
#pragma unroll
      for (int i = 0; i < 32; ++i)
        if (i < nu) Kk[i * ld + cc] = v[i];
    } else {
      T* dst = wHi + (int64_t)k * nu * nu;
#pragma unroll
      for (int i = 0; i < 32; ++i)
        if (i < nu) dst[i * ld + cc] = (T)v[i];
    }
  }
  __syncthreads();
  // P_k = Q + sigma I + A_k' P A_k + G_k' K_k, symmetrised as (P_k + P_k')/2:
  // one thread owns the pair (i, j), (j, i) and overwrites P (P_{k+1} is dead).
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    if (update_P && j >= i) {
      const D a0 = ((i == j) ? (D)q[i] + sc.sigma + state_rho<D>(in, d, i, sc) : 0.0) +
                   contact_weight<D>(in, d, k, i, j, sc);
      D a1 = blocked_sum<D>(0, 1, nx, [&](int t) { return Ak[t * nx + i] * PA[t * nx + j]; }, a0);
      D a2 = blocked_sum<D>(0, 1, nx, [&](int t) { return Ak[t * nx + j] * PA[t * nx + i]; }, a0);
      a1 = blocked_sum<D>(0, 1, nu, [&](int t) { return G[t * nx + i] * Kk[t * nx + j]; }, a1);
      a2 = blocked_sum<D>(0, 1, nu, [&](int t) { return G[t * nx + j] * Kk[t * nx + i]; }, a2);
      const D v = 0.5 * (a1 + a2);
      P[i * nx + j] = v;
      P[j * nx + i] = v;
    }
    const D acl = blocked_sum<D>(0, 1, nu, [&](int t) { return Bk[i * nu + t] * Kk[t * nx + j]; }, Ak[idx]);
    wAcl[(int64_t)k * nx * nx + idx] = (T)acl;
  }
  for (int idx = tid; idx < nu * nx; idx += nt) wK[(int64_t)k * nu * nx + idx] = (T)Kk[idx];
  __syncthreads();
  return true;
}

}  // namespace mpc
