// Device helpers for the per-stage constraint rows C_k = [I_nu ; friction pyramid].
//
// Row layout (m = nu + 4 n_feet rows per stage):
//   rows 0 .. n_tau-1              torque box            [-tau_max, tau_max]
//   rows n_tau + f*fd + j          foot f, component j   stance: f_z >= 0, others free
//                                                        swing : [0, 0]
//   rows nu + 4f + {0,1,2,3}       pyramid facets of f   f_x - mu f_z, -f_x - mu f_z,
//                                                        f_y - mu f_z, -f_y - mu f_z
//                                                        stance: <= 0, swing: free
// These are the contact and swing conditions of Eq. (mpc_formulation) with the
// friction cone replaced by its 4-sided outer pyramid.  The penalty of a row is
// rho, rho_eq_scale * rho for equality rows (l == h) and rho_min for rows with
// both bounds infinite (OSQP's choice, adopted in Sec. III-B).  The four facets
// of one foot always share a penalty, so C_k' diag(rho) C_k is diagonal.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "mpc_internal.h"

namespace mpc {

template <typename T>
__device__ inline T pos_inf() {
  return (T)INFINITY;
}

// Bounds and penalty of row i at a stage with stance flags st (n_feet bytes).
template <typename T, typename TT>
__device__ inline void row_bounds(const AgentDesc& d, int i, const uint8_t* st, const TT* tau,
                                  const SolverConsts& sc, T& lo, T& hi, T& rho) {
  const T inf = pos_inf<T>();
  if (i < d.n_tau) {
    lo = -(T)tau[i];
    hi = (T)tau[i];
  } else if (i < d.nu) {
    const int f = (i - d.n_tau) / d.foot_dim, j = (i - d.n_tau) % d.foot_dim;
    if (st[f]) {
      lo = (j == 2) ? (T)0 : -inf;
      hi = inf;
    } else {
      lo = (T)0;
      hi = (T)0;
    }
  } else {
    const int f = (i - d.nu) >> 2;
    lo = -inf;
    hi = st[f] ? (T)0 : inf;
  }
  if (lo == hi)
    rho = (T)(sc.rho_eq * sc.rho);
  else if (isinf(lo) && isinf(hi))
    rho = (T)sc.rho_min;
  else
    rho = (T)sc.rho;
}

// Penalty of the joint-limit row of state component i (0 without limits):
// rho_eq_scale * rho for an equality, rho_min with both bounds infinite, rho
// otherwise -- the penalty rule of the input rows.
template <typename T, typename TT>
__device__ inline T state_rho(const Inputs<TT>& in, const AgentDesc& d, int i, const SolverConsts& sc) {
  if (!in.xlo) return (T)0;
  const TT lo = in.xlo[d.oq + i], hi = in.xhi[d.oq + i];
  if (lo == hi) return (T)(sc.rho_eq * sc.rho);
  if (isinf(lo) && isinf(hi)) return (T)sc.rho_min;
  return (T)sc.rho;
}

// No-slip row `row` (foot row / foot_dim) of state x_k, k = 1..N: an equality
// J_f v_k = 0 while the foot is in stance at stage min(k, N-1) (penalty
// rho_eq_scale * rho), a free row while it swings (rho_min).  Returns whether
// the row is an equality; rho receives its penalty.
__device__ inline bool contact_row(const AgentDesc& d, const uint8_t* stance, int k, int row,
                                   const SolverConsts& sc, double& rho) {
  const int sk = k < d.N ? k : d.N - 1;
  const bool eq = stance[sk * d.n_feet + row / d.foot_dim] != 0;
  rho = eq ? sc.rho_eq * sc.rho : sc.rho_min;
  return eq;
}

// Entry (i, j) of Jc' diag(rho_c,k) Jc, the no-slip rows' term in the state
// weight of stage k (0 without the rows or at k = 0).
template <typename T, typename TT>
__device__ inline T contact_weight(const Inputs<TT>& in, const AgentDesc& d, int k, int i, int j,
                                   const SolverConsts& sc) {
  if (!in.J || k == 0) return (T)0;
  const TT* Jc = in.J + d.oJ;
  const uint8_t* stance = in.st + d.ost;
  const int nc = d.n_feet * d.foot_dim;
  T acc = 0;
  for (int row = 0; row < nc; ++row) {
    double rr;
    contact_row(d, stance, k, row, sc, rr);
    acc += (T)Jc[row * d.nx + i] * (T)rr * (T)Jc[row * d.nx + j];
  }
  return acc;
}

// Diagonal of R + sigma I + C' diag(rho) C for input j (rho = this stage's row penalties).
template <typename T, typename R>
__device__ inline T rtilde_diag(const AgentDesc& d, int j, T rj, T mu, const R* rho,
                                const SolverConsts& sc) {
  T v = rj + (T)sc.sigma + (T)rho[j];
  if (j >= d.n_tau) {
    const int f = (j - d.n_tau) / d.foot_dim, c = (j - d.n_tau) % d.foot_dim;
    const R* rp = rho + d.nu + 4 * f;
    if (c == 0) v += (T)rp[0] + (T)rp[1];
    if (c == 1) v += (T)rp[2] + (T)rp[3];
    if (c == 2) v += mu * mu * ((T)rp[0] + (T)rp[1] + (T)rp[2] + (T)rp[3]);
  }
  return v;
}

// (C' w)_j for one stage (w has m entries).
template <typename T>
__device__ inline T ct_row(const AgentDesc& d, int j, T mu, const T* w) {
  T v = w[j];
  if (j >= d.n_tau) {
    const int f = (j - d.n_tau) / d.foot_dim, c = (j - d.n_tau) % d.foot_dim;
    const T* wp = w + d.nu + 4 * f;
    if (c == 0) v += wp[0] - wp[1];
    if (c == 1) v += wp[2] - wp[3];
    if (c == 2) v -= mu * (wp[0] + wp[1] + wp[2] + wp[3]);
  }
  return v;
}

// (C u)_i for one stage.
template <typename T>
__device__ inline T c_row(const AgentDesc& d, int i, T mu, const T* u) {
  if (i < d.nu) return u[i];
  const int f = (i - d.nu) >> 2, p = (i - d.nu) & 3;
  const int b = d.n_tau + f * d.foot_dim;
  const T fz = u[b + 2];
  const T t = (p < 2) ? u[b] : u[b + 1];
  return ((p & 1) ? -t : t) - mu * fz;
}

}  // namespace mpc
