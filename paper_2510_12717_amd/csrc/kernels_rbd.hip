// The real-time iteration's front and back end on the GPU (Alg. 1's f_KKT and
// f_RNEA): rigid-body dynamics of a kinematic tree, in FP64.
//
//   k_rnea        : inverse dynamics (Eq. (rnea)) M(q) qdd + h(q, qd) - J(q)' F,
//                   one thread per configuration;
//   k_linearize   : the QP data of every stage of every agent, A_k = df/dx and
//                   B_k = df/du of the semi-implicit Euler step of
//                   Eq. (mpc_formulation) by central differences, one thread
//                   per (agent, stage, column) evaluating the step twice, and
//                   f(x_k, u_k) itself; k_lin_offset then forms
//                   c_k = f(x_k, u_k) - A_k x_k - B_k u_k;
//   k_rti_torque  : Eq. (mpc_torque), tau = Kp (q* - q) + Kd (qd* - qd) + tau_rnea
//                   for the joints, tau_rnea from the first stage of the QP
//                   solution (qdd* = (qd*_1 - qd*_0) / dt, F* = the wrench part of u*_0).
//
// Spatial vectors are (angular, linear).  A body's transform from its parent
// is kept as (E, r): E maps parent coordinates to body coordinates, r is the
// body origin in parent coordinates; motion vectors transform as
// (E w, E (v - r x w)), forces back to the parent as (E'n + r x E'f, E'f).
// The floating base is the first six joints (three prismatic along the world
// axes, three revolute), so every coordinate is additive.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/mpc.h"
#include "host_api.h"
#include "rbd.h"

namespace mpc {

namespace {

struct V3 {
  double x, y, z;
};
__device__ inline V3 v3(double a, double b, double c) { return V3{a, b, c}; }
__device__ inline V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
struct M3 {
  double m[9];  // row-major
};
__device__ inline V3 mul(const M3& E, V3 a) {
  return v3(E.m[0] * a.x + E.m[1] * a.y + E.m[2] * a.z, E.m[3] * a.x + E.m[4] * a.y + E.m[5] * a.z,
            E.m[6] * a.x + E.m[7] * a.y + E.m[8] * a.z);
}
__device__ inline V3 mulT(const M3& E, V3 a) {
  return v3(E.m[0] * a.x + E.m[3] * a.y + E.m[6] * a.z, E.m[1] * a.x + E.m[4] * a.y + E.m[7] * a.z,
            E.m[2] * a.x + E.m[5] * a.y + E.m[8] * a.z);
}
__device__ inline M3 mulM(const M3& A, const M3& B) {
  M3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
__device__ inline V3 ld3(const double* p) { return v3(p[0], p[1], p[2]); }

// Rotation by th about the unit axis a (body axes in parent coordinates), its
// transpose being the parent-to-body map.
__device__ inline M3 axis_rotation(V3 a, double th) {
  const double s = sin(th), c = cos(th), t = 1.0 - c;
  M3 R;
  R.m[0] = c + t * a.x * a.x;
  R.m[1] = t * a.x * a.y - s * a.z;
  R.m[2] = t * a.x * a.z + s * a.y;
  R.m[3] = t * a.y * a.x + s * a.z;
  R.m[4] = c + t * a.y * a.y;
  R.m[5] = t * a.y * a.z - s * a.x;
  R.m[6] = t * a.z * a.x - s * a.y;
  R.m[7] = t * a.z * a.y + s * a.x;
  R.m[8] = c + t * a.z * a.z;
  return R;
}

// Per-body transform from the parent (E, r) at joint value qi.
__device__ inline void joint_xform(const ModelDev& md, int i, double qi, M3& E, V3& r) {
  const V3 a = ld3(md.axis + 3 * i), off = ld3(md.offset + 3 * i);
  if (md.jtype[i] == 1) {
    for (int k = 0; k < 9; ++k) E.m[k] = (k % 4 == 0) ? 1.0 : 0.0;
    r = off + qi * a;
  } else {
    const M3 R = axis_rotation(a, qi);
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) E.m[3 * u + v] = R.m[3 * v + u];
    r = off;
  }
}

// I (w, v) for the body inertia (m, c, Ic principal): linear m (v - c x w),
// angular Ic w + c x linear.
__device__ inline void inertia_apply(const ModelDev& md, int i, V3 w, V3 v, V3& n, V3& f) {
  const double m = md.mass[i];
  const V3 c = ld3(md.com + 3 * i), I = ld3(md.inertia + 3 * i);
  f = m * (v - cross(c, w));
  n = v3(I.x * w.x, I.y * w.y, I.z * w.z) + cross(c, f);
}

// Inverse dynamics of one configuration; tau[n] out.  F (nullable): foot
// wrenches, world frame, at the contact points.  Scratch: per-body transforms,
// velocities, accelerations and forces (private memory).
__device__ void rnea_dev(const ModelDev& md, const double* q, const double* qd, const double* qdd,
                         const double* F, double* tau) {
  const int n = md.n;
  M3 E[kMaxBodies];
  V3 r[kMaxBodies];
  V3 w[kMaxBodies], v[kMaxBodies], aw[kMaxBodies], av[kMaxBodies], fn[kMaxBodies], ff[kMaxBodies];
  M3 E0[kMaxBodies];  // world-to-body rotation
  V3 p0[kMaxBodies];  // body origin, world
  for (int i = 0; i < n; ++i) {
    joint_xform(md, i, q[i], E[i], r[i]);
    const int par = md.parent[i];
    V3 wp = v3(0, 0, 0), vp = v3(0, 0, 0), awp = v3(0, 0, 0), avp = v3(0, 0, md.gravity);
    if (par >= 0) {
      wp = w[par];
      vp = v[par];
      awp = aw[par];
      avp = av[par];
      E0[i] = mulM(E[i], E0[par]);
      p0[i] = p0[par] + mulT(E0[par], r[i]);
    } else {
      E0[i] = E[i];
      p0[i] = r[i];
    }
    // X (w, v) = (E w, E (v - r x w))
    V3 wi = mul(E[i], wp), vi = mul(E[i], vp - cross(r[i], wp));
    V3 awi = mul(E[i], awp), avi = mul(E[i], avp - cross(r[i], awp));
    const V3 ax = ld3(md.axis + 3 * i);
    const bool pri = md.jtype[i] == 1;
    // S qd: (ax qd, 0) revolute, (0, ax qd) prismatic
    const V3 sw = pri ? v3(0, 0, 0) : qd[i] * ax, sv = pri ? qd[i] * ax : v3(0, 0, 0);
    wi = wi + sw;
    vi = vi + sv;
    // a = X a_p + S qdd + v x (S qd)
    const V3 cw = cross(wi, sw), cv = cross(vi, sw) + cross(wi, sv);
    awi = awi + (pri ? v3(0, 0, 0) : qdd[i] * ax) + cw;
    avi = avi + (pri ? qdd[i] * ax : v3(0, 0, 0)) + cv;
    w[i] = wi;
    v[i] = vi;
    aw[i] = awi;
    av[i] = avi;
    // f = I a + v x* I v
    V3 n1, f1, n2, f2;
    inertia_apply(md, i, awi, avi, n1, f1);
    inertia_apply(md, i, wi, vi, n2, f2);
    fn[i] = n1 + cross(wi, n2) + cross(vi, f2);
    ff[i] = f1 + cross(wi, f2);
  }
  if (F) {
    for (int f = 0; f < md.n_feet; ++f) {
      const int b = md.foot_body[f];
      const V3 pt = p0[b] + mulT(E0[b], ld3(md.foot_offset + 3 * f));
      const V3 fw = ld3(F + f * md.foot_dim);
      const V3 nw = md.foot_dim == 6 ? ld3(F + f * md.foot_dim + 3) : v3(0, 0, 0);
      // world wrench about the body origin, into body axes
      fn[b] = fn[b] - mul(E0[b], nw + cross(pt - p0[b], fw));
      ff[b] = ff[b] - mul(E0[b], fw);
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    const V3 ax = ld3(md.axis + 3 * i);
    tau[i] = md.jtype[i] == 1 ? dot(ax, ff[i]) : dot(ax, fn[i]);
    const int par = md.parent[i];
    if (par >= 0) {
      const V3 fp = mulT(E[i], ff[i]);
      fn[par] = fn[par] + mulT(E[i], fn[i]) + cross(r[i], fp);
      ff[par] = ff[par] + fp;
    }
  }
}

// Spatial inertia (6x6, row-major) of body i at its origin.
__device__ inline void inertia6(const ModelDev& md, int i, double* I) {
  const double m = md.mass[i];
  const V3 c = ld3(md.com + 3 * i), J = ld3(md.inertia + 3 * i);
  const double C[9] = {0, -c.z, c.y, c.z, 0, -c.x, -c.y, c.x, 0};
  for (int u = 0; u < 3; ++u)
    for (int v = 0; v < 3; ++v) {
      double cc = 0;  // (C C')_uv
      for (int t = 0; t < 3; ++t) cc += C[3 * u + t] * C[3 * v + t];
      I[6 * u + v] = (u == v ? (u == 0 ? J.x : u == 1 ? J.y : J.z) : 0.0) + m * cc;
      I[6 * u + 3 + v] = m * C[3 * u + v];
      I[6 * (3 + u) + v] = m * C[3 * v + u];
      I[6 * (3 + u) + 3 + v] = u == v ? m : 0.0;
    }
}

// 6x6 motion transform of (E, r): [E 0; -E r^ E].
__device__ inline void xform6(const M3& E, V3 r, double* X) {
  const double R[9] = {0, -r.z, r.y, r.z, 0, -r.x, -r.y, r.x, 0};
  for (int u = 0; u < 3; ++u)
    for (int v = 0; v < 3; ++v) {
      double er = 0;
      for (int t = 0; t < 3; ++t) er += E.m[3 * u + t] * R[3 * t + v];
      X[6 * u + v] = E.m[3 * u + v];
      X[6 * u + 3 + v] = 0.0;
      X[6 * (3 + u) + v] = -er;
      X[6 * (3 + u) + 3 + v] = E.m[3 * u + v];
    }
}

// Mass matrix by the composite-rigid-body algorithm into M (n x n, row-major).
// Transforms are kept as (E, r) and expanded to 6x6 one at a time.
__device__ void crba_dev(const ModelDev& md, const double* q, double* M) {
  const int n = md.n;
  double Ic[kMaxBodies][36];
  M3 Eb[kMaxBodies];
  V3 rb[kMaxBodies];
  for (int i = 0; i < n; ++i) {
    joint_xform(md, i, q[i], Eb[i], rb[i]);
    inertia6(md, i, Ic[i]);
  }
  // bodies on different branches couple through no joint: their entries stay 0
  for (int k = 0; k < n * n; ++k) M[k] = 0.0;
  double X[36];
  for (int i = n - 1; i >= 0; --i) {
    const int par = md.parent[i];
    if (par < 0) continue;
    xform6(Eb[i], rb[i], X);
    // Ic_par += X' Ic X
    double T[36];
    for (int u = 0; u < 6; ++u)
      for (int v = 0; v < 6; ++v) {
        double s = 0;
        for (int t = 0; t < 6; ++t) s += Ic[i][6 * u + t] * X[6 * t + v];
        T[6 * u + v] = s;
      }
    for (int u = 0; u < 6; ++u)
      for (int v = 0; v < 6; ++v) {
        double s = 0;
        for (int t = 0; t < 6; ++t) s += X[6 * t + u] * T[6 * t + v];
        Ic[par][6 * u + v] += s;
      }
  }
  for (int i = n - 1; i >= 0; --i) {
    double S[6] = {0, 0, 0, 0, 0, 0};
    const V3 ax = ld3(md.axis + 3 * i);
    const int o = md.jtype[i] == 1 ? 3 : 0;
    S[o] = ax.x;
    S[o + 1] = ax.y;
    S[o + 2] = ax.z;
    // F = Ic S as a force (n, f), carried to the ancestors by X' (n, f) =
    // (E'n + r x E'f, E'f)
    V3 fn = v3(0, 0, 0), ff = v3(0, 0, 0);
    {
      double Fv[6];
      for (int u = 0; u < 6; ++u) {
        double s = 0;
        for (int t = 0; t < 6; ++t) s += Ic[i][6 * u + t] * S[t];
        Fv[u] = s;
      }
      fn = v3(Fv[0], Fv[1], Fv[2]);
      ff = v3(Fv[3], Fv[4], Fv[5]);
    }
    M[i * n + i] = md.jtype[i] == 1 ? dot(ax, ff) : dot(ax, fn);
    int j = i;
    while (md.parent[j] >= 0) {
      const V3 fp = mulT(Eb[j], ff);
      fn = mulT(Eb[j], fn) + cross(rb[j], fp);
      ff = fp;
      j = md.parent[j];
      const V3 aj = ld3(md.axis + 3 * j);
      const double mij = md.jtype[j] == 1 ? dot(aj, ff) : dot(aj, fn);
      M[i * n + j] = mij;
      M[j * n + i] = mij;
    }
  }
}

// Semi-implicit Euler step f(x, u) into xn (x = (q, qd), u = (joint torques,
// foot wrenches)).  Returns false if M is not positive definite.
__device__ bool step_dev(const ModelDev& md, const double* x, const double* u, double dt, double* xn) {
  const int n = md.n, nj = md.n - 6;
  double M[kMaxBodies * kMaxBodies];
  double b[kMaxBodies], z[kMaxBodies];
  for (int i = 0; i < n; ++i) z[i] = 0.0;
  crba_dev(md, x, M);
  // b = S' tau - (h - J'F) = S' tau - rnea(q, qd, 0, F)
  rnea_dev(md, x, x + n, z, u + nj, b);
  for (int i = 0; i < n; ++i) b[i] = (i >= 6 ? u[i - 6] : 0.0) - b[i];
  // Cholesky M = L L' in place (lower), then two substitutions
  for (int j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int t = 0; t < j; ++t) s -= M[j * n + t] * M[j * n + t];
    if (!(s > 0.0)) return false;
    const double l = sqrt(s);
    M[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double v = M[i * n + j];
      for (int t = 0; t < j; ++t) v -= M[i * n + t] * M[j * n + t];
      M[i * n + j] = v / l;
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int t = 0; t < i; ++t) s -= M[i * n + t] * b[t];
    b[i] = s / M[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int t = i + 1; t < n; ++t) s -= M[t * n + i] * b[t];
    b[i] = s / M[i * n + i];
  }
  for (int i = 0; i < n; ++i) {
    const double qd1 = x[n + i] + dt * b[i];
    xn[n + i] = qd1;
    xn[i] = x[i] + dt * qd1;
  }
  return true;
}

__global__ void __launch_bounds__(64)
k_rnea(ModelDev md, int count, const double* __restrict__ q, const double* __restrict__ qd,
       const double* __restrict__ qdd, const double* __restrict__ F, double* __restrict__ tau) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int n = md.n, nf = md.n_feet * md.foot_dim;
  rnea_dev(md, q + (int64_t)t * n, qd + (int64_t)t * n, qdd + (int64_t)t * n,
           F ? F + (int64_t)t * nf : nullptr, tau + (int64_t)t * n);
}

// Thread (agent, stage, column j): column j < nx + nu of A_k | B_k by central
// differences with step h; column nx + nu: f(x_k, u_k) itself, into c.
__global__ void __launch_bounds__(64)
k_linearize(ModelDev md, int n_agents, int N, double dt, double h, const double* __restrict__ X,
            const double* __restrict__ U, double* __restrict__ A, double* __restrict__ B,
            double* __restrict__ C, int32_t* __restrict__ status) {
  const int nx = 2 * md.n, nu = md.n - 6 + md.n_feet * md.foot_dim, ncol = nx + nu + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_agents * N * ncol) return;
  const int j = (int)(t % ncol);
  const int64_t ak = t / ncol;  // agent * N + stage
  const double* x = X + ak * nx;
  const double* u = U + ak * nu;
  double xp[2 * kMaxBodies], up[kMaxU], fp[2 * kMaxBodies], fm[2 * kMaxBodies];
  bool finite = true;
  for (int i = 0; i < nx; ++i) {
    xp[i] = x[i];
    finite = finite && isfinite(xp[i]);
  }
  for (int i = 0; i < nu; ++i) {
    up[i] = u[i];
    finite = finite && isfinite(up[i]);
  }
  // one call site of the step (two evaluations for a column, one for f), so
  // that the step's private arrays exist once
  const bool value = j == nx + nu;
  double* var = value ? nullptr : (j < nx ? xp + j : up + (j - nx));
  const double v0 = value ? 0.0 : *var;
  bool ok = true;
  for (int e = 0; e < (value ? 1 : 2); ++e) {
    if (!value) *var = e == 0 ? v0 + h : v0 - h;
    ok = step_dev(md, xp, up, dt, e == 0 ? fp : fm) && ok;
  }
  if (value) {
    for (int i = 0; i < nx; ++i) C[ak * nx + i] = fp[i];
  } else {
    const double ih = 0.5 / h;
    if (j < nx)
      for (int i = 0; i < nx; ++i) A[(ak * nx + i) * nx + j] = (fp[i] - fm[i]) * ih;
    else
      for (int i = 0; i < nx; ++i) B[(ak * nx + i) * nu + (j - nx)] = (fp[i] - fm[i]) * ih;
  }
  // a non-finite point outranks a failed factorisation, whichever thread of
  // the agent writes last
  if (!finite) atomicMax(status + ak / N, (int32_t)AGENT_NONFINITE);
  else if (!ok) atomicMax(status + ak / N, (int32_t)AGENT_NOT_PD);
}

// c_k = f(x_k, u_k) - A_k x_k - B_k u_k (C holds f(x_k, u_k) on entry).
__global__ void __launch_bounds__(64)
k_lin_offset(int nx, int nu, int64_t rows, const double* __restrict__ X, const double* __restrict__ U,
             const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows) return;
  const int64_t ak = t / nx;
  const int i = (int)(t % nx);
  const double* x = X + ak * nx;
  const double* u = U + ak * nu;
  double s = C[t];
  for (int k = 0; k < nx; ++k) s -= A[(ak * nx + i) * nx + k] * x[k];
  for (int k = 0; k < nu; ++k) s -= B[(ak * nx + i) * nu + k] * u[k];
  C[t] = s;
}

__global__ void __launch_bounds__(64)
k_rti_torque(ModelDev md, int count, double dt, double kp, double kd, const double* __restrict__ x0,
             const double* __restrict__ x1, const double* __restrict__ u0,
             const double* __restrict__ qm, const double* __restrict__ qdm, double* __restrict__ tau) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int n = md.n, nx = 2 * n, nj = n - 6, nu = nj + md.n_feet * md.foot_dim;
  const double* a = x0 + (int64_t)t * nx;
  const double* b = x1 + (int64_t)t * nx;
  double qdd[kMaxBodies], tr[kMaxBodies];
  for (int i = 0; i < n; ++i) qdd[i] = (b[n + i] - a[n + i]) / dt;
  rnea_dev(md, a, a + n, qdd, u0 + (int64_t)t * nu + nj, tr);
  for (int i = 0; i < nj; ++i)
    tau[(int64_t)t * nj + i] = kp * (a[6 + i] - qm[(int64_t)t * n + 6 + i]) +
                               kd * (a[n + 6 + i] - qdm[(int64_t)t * n + 6 + i]) + tr[6 + i];
}

}  // namespace

hipError_t launch_rnea(const ModelDev& md, int count, const double* q, const double* qd,
                       const double* qdd, const double* F, double* tau, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rnea, dim3((count + 63) / 64), dim3(64), 0, s, md, count, q, qd, qdd, F, tau);
  return hipGetLastError();
}

hipError_t launch_linearize(const ModelDev& md, int n_agents, int N, double dt, const double* X,
                            const double* U, double* A, double* B, double* C, int32_t* status,
                            hipStream_t s) {
  const int nx = 2 * md.n, nu = md.n - 6 + md.n_feet * md.foot_dim;
  const int64_t threads = (int64_t)n_agents * N * (nx + nu + 1);
  if (threads <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_linearize, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, md, n_agents, N,
                     dt, 1e-5, X, U, A, B, C, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t rows = (int64_t)n_agents * N * nx;
  hipLaunchKernelGGL(k_lin_offset, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, s, nx, nu, rows, X, U,
                     A, B, C);
  return hipGetLastError();
}

hipError_t launch_rti_torque(const ModelDev& md, int count, double dt, double kp, double kd,
                             const double* x0, const double* x1, const double* u0, const double* qm,
                             const double* qdm, double* tau, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rti_torque, dim3((count + 63) / 64), dim3(64), 0, s, md, count, dt, kp, kd, x0,
                     x1, u0, qm, qdm, tau);
  return hipGetLastError();
}

}  // namespace mpc

// ------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------

struct mpc_model_s {
  int device = 0;
  mpc::ModelDev md{};
  void* buf = nullptr;  // one device allocation holding every array
};

extern "C" mpc_status mpc_model_create(const mpc_model_desc* d, int32_t device, mpc_model_t* out) {
  using namespace mpc;
  if (!d || !out) return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const int n = d->n_bodies, nf = d->n_feet;
  if (n < 7 || n > kMaxBodies || nf < 0 || nf > 8 || (d->foot_dim != 3 && d->foot_dim != 6) ||
      n - 6 + nf * d->foot_dim > kMaxU || !(d->gravity >= 0))
    return api_fail(MPC_ERR_UNSUPPORTED_SHAPE,
                    "model: 7..24 bodies (six base coordinates first), at most 8 feet of 3 or 6 "
                    "wrench components, joints + wrench components <= 32");
  if (!d->parent || !d->joint_type || !d->axis || !d->offset || !d->mass || !d->com || !d->inertia ||
      (nf > 0 && (!d->foot_body || !d->foot_offset)))
    return api_fail(MPC_ERR_INVALID_ARG, "null model array");
  for (int i = 0; i < n; ++i) {
    const bool base = i < 6;
    if (d->parent[i] != i - 1 && (base || d->parent[i] < 5 || d->parent[i] >= i))
      return api_fail(MPC_ERR_INVALID_ARG,
                      "model: bodies in topological order, the first six a chain (the floating "
                      "base), every other body's parent an earlier body from the sixth on");
    if (d->joint_type[i] != 0 && d->joint_type[i] != 1)
      return api_fail(MPC_ERR_INVALID_ARG, "model: joint type 0 (revolute) or 1 (prismatic)");
    const double* a = d->axis + 3 * i;
    if (!(std::fabs(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] - 1.0) < 1e-9))
      return api_fail(MPC_ERR_INVALID_ARG, "model: joint axes must be unit vectors");
  }
  // the first five bodies are the floating base's massless intermediate
  // frames; the base body (the sixth) and every limb carry mass
  for (int i = 0; i < n; ++i) {
    const double lo = i < 5 ? -0.0 : 0.0;
    bool ok = std::isfinite(d->mass[i]) && (i < 5 ? d->mass[i] >= lo : d->mass[i] > lo);
    for (int t = 0; t < 3; ++t) {
      const double v = d->inertia[3 * i + t];
      ok = ok && std::isfinite(v) && (i < 5 ? v >= lo : v > lo);
    }
    if (!ok)
      return api_fail(MPC_ERR_INVALID_ARG,
                      "model: every body from the sixth on needs a positive mass and inertia, "
                      "the first five a non-negative one");
  }
  for (int f = 0; f < nf; ++f)
    if (d->foot_body[f] < 6 || d->foot_body[f] >= n)
      return api_fail(MPC_ERR_INVALID_ARG, "model: a foot on a body past the base");
  MPC_HIP_TRY(hipSetDevice(device));
  const size_t dbl = (size_t)n * (3 + 3 + 1 + 3 + 3) + (size_t)nf * 3;
  const size_t ints = (size_t)n * 2 + (size_t)nf;
  std::vector<unsigned char> host(8 * dbl + 4 * ints);
  double* hd = reinterpret_cast<double*>(host.data());
  int32_t* hi = reinterpret_cast<int32_t*>(host.data() + 8 * dbl);
  size_t o = 0;
  auto putd = [&](const double* src, size_t k) {
    const size_t at = o;
    for (size_t t = 0; t < k; ++t) hd[o + t] = src[t];
    o += k;
    return at;
  };
  const size_t oa = putd(d->axis, 3 * n), oo = putd(d->offset, 3 * n), om = putd(d->mass, n),
               oc = putd(d->com, 3 * n), oi = putd(d->inertia, 3 * n),
               of = nf ? putd(d->foot_offset, 3 * nf) : o;
  for (int i = 0; i < n; ++i) {
    hi[i] = d->parent[i];
    hi[n + i] = d->joint_type[i];
  }
  for (int f = 0; f < nf; ++f) hi[2 * n + f] = d->foot_body[f];
  auto* m = new mpc_model_s();
  m->device = device;
  hipError_t e = hipMalloc(&m->buf, host.size());
  if (e == hipSuccess) e = hipMemcpy(m->buf, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(m->buf);
    delete m;
    return api_fail(e == hipErrorOutOfMemory ? MPC_ERR_OUT_OF_MEMORY : MPC_ERR_HIP,
                    std::string("model upload: ") + hipGetErrorString(e));
  }
  const double* dd = reinterpret_cast<const double*>(m->buf);
  const int32_t* di = reinterpret_cast<const int32_t*>((const unsigned char*)m->buf + 8 * dbl);
  m->md = ModelDev{n, nf, d->foot_dim, d->gravity, di, di + n, dd + oa, dd + oo, dd + om, dd + oc, dd + oi,
                   nf ? di + 2 * n : nullptr, nf ? dd + of : nullptr};
  *out = m;
  return MPC_OK;
}

extern "C" mpc_status mpc_model_destroy(mpc_model_t m) {
  if (!m) return mpc::api_fail(MPC_ERR_INVALID_ARG, "null model");
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  hipFree(m->buf);
  delete m;
  return MPC_OK;
}

extern "C" mpc_status mpc_rnea(mpc_model_t m, int32_t count, const double* q, const double* qd,
                               const double* qdd, const double* F, double* tau, void* stream) {
  using namespace mpc;
  if (!m || count < 0 || (count > 0 && (!q || !qd || !qdd || !tau)))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  MPC_HIP_TRY(hipSetDevice(m->device));
  MPC_HIP_TRY(launch_rnea(m->md, count, q, qd, qdd, F, tau, (hipStream_t)stream));
  return MPC_OK;
}

extern "C" mpc_status mpc_linearize(mpc_model_t m, int32_t n_agents, int32_t N, double dt,
                                    const double* x, const double* u, double* A, double* B, double* c,
                                    int32_t* status, void* stream) {
  using namespace mpc;
  if (!m || n_agents < 0 || N < 1 || N > 64 || !(dt > 0))
    return api_fail(MPC_ERR_INVALID_ARG, "n_agents >= 0, 1 <= N <= 64 and dt > 0 required");
  if (n_agents > 0 && (!x || !u || !A || !B || !c || !status))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  MPC_HIP_TRY(hipSetDevice(m->device));
  MPC_HIP_TRY(launch_linearize(m->md, n_agents, N, dt, x, u, A, B, c, status, (hipStream_t)stream));
  return MPC_OK;
}

extern "C" mpc_status mpc_rti_torque(mpc_model_t m, int32_t count, double dt, double kp, double kd,
                                     const double* x0, const double* x1, const double* u0,
                                     const double* q, const double* qd, double* tau, void* stream) {
  using namespace mpc;
  if (!m || count < 0 || !(dt > 0) ||
      (count > 0 && (!x0 || !x1 || !u0 || !q || !qd || !tau)))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument, or dt <= 0");
  MPC_HIP_TRY(hipSetDevice(m->device));
  MPC_HIP_TRY(launch_rti_torque(m->md, count, dt, kp, kd, x0, x1, u0, q, qd, tau, (hipStream_t)stream));
  return MPC_OK;
}
