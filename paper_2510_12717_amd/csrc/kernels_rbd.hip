// The real-time iteration's front and back end on the GPU (Alg. 1's f_KKT and
// f_RNEA): rigid-body dynamics of a kinematic tree, in FP64.
//
//   k_rnea        : inverse dynamics (Eq. (rnea)) M(q) qdd + h(q, qd) - J(q)' F,
//                   one thread per configuration;
//   k_linearize   : the QP data of every stage of every agent, A_k = df/dx,
//                   B_k = df/du and c_k = f(x_k, u_k) - A_k x_k - B_k u_k of the
//                   semi-implicit Euler step of Eq. (mpc_formulation), one
//                   workgroup per (agent, stage): mass matrix, forward dynamics
//                   and the derivatives of inverse dynamics in closed form from
//                   the tree's world-frame composite quantities, in LDS;
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

// ---- world-frame spatial algebra for the linearisation -----------------------
// A 6-vector is (angular, linear) for motions and (moment, force) for forces,
// all about the world origin.
struct S6 {
  V3 a, b;
};
__device__ inline S6 s6(V3 a, V3 b) { return S6{a, b}; }
__device__ inline S6 operator+(S6 x, S6 y) { return s6(x.a + y.a, x.b + y.b); }
__device__ inline S6 operator-(S6 x, S6 y) { return s6(x.a - y.a, x.b - y.b); }
__device__ inline S6 operator*(double t, S6 x) { return s6(t * x.a, t * x.b); }
__device__ inline S6 ld6(const double* p) { return s6(ld3(p), ld3(p + 3)); }
__device__ inline void st6(double* p, S6 x) {
  p[0] = x.a.x; p[1] = x.a.y; p[2] = x.a.z;
  p[3] = x.b.x; p[4] = x.b.y; p[5] = x.b.z;
}
// m x n (motion on motion) and m x* f (motion on force)
__device__ inline S6 crm(S6 m, S6 n) { return s6(cross(m.a, n.a), cross(m.a, n.b) + cross(m.b, n.a)); }
__device__ inline S6 crf(S6 m, S6 f) { return s6(cross(m.a, f.a) + cross(m.b, f.b), cross(m.a, f.b)); }
__device__ inline double dot6(S6 m, S6 f) { return dot(m.a, f.a) + dot(m.b, f.b); }
// 6x6 row-major matrix times a 6-vector
__device__ inline S6 mul6(const double* M, S6 x) {
  const double in[6] = {x.a.x, x.a.y, x.a.z, x.b.x, x.b.y, x.b.z};
  double o[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) t += M[6 * r + c] * in[c];
    o[r] = t;
  }
  return s6(v3(o[0], o[1], o[2]), v3(o[3], o[4], o[5]));
}

// Body i's placement relative to its parent at joint value qi: rotation (body
// axes in parent coordinates) and origin.
__device__ inline void joint_local(const ModelDev& md, int i, double qi, M3& R, V3& p) {
  const V3 a = ld3(md.axis + 3 * i), off = ld3(md.offset + 3 * i);
  if (md.jtype[i] == 1) {
    for (int k = 0; k < 9; ++k) R.m[k] = (k % 4 == 0) ? 1.0 : 0.0;
    p = off + qi * a;
  } else {
    R = axis_rotation(a, qi);
    p = off;
  }
}

constexpr int kLinThreads = 128;
constexpr int kMaxCols = 2 * kMaxBodies + kMaxU;  // x and u columns
constexpr int kMaxFeet = 8;

// Shared state of one stage's linearisation (world frame, per body).
struct LinLds {
  double S[kMaxBodies][6];      // joint motion subspace
  double v[kMaxBodies][6];      // velocity
  double a[kMaxBodies][6];      // acceleration: qdd = 0 first, then qdd = qdd0
  double Io[kMaxBodies][36];    // own spatial inertia
  double IC[kMaxBodies][36];    // composite inertia of the subtree
  double BC[kMaxBodies][36];    // composite of v x* I - I v x
  double hC[kMaxBodies][6];     // composite momentum
  double fC[kMaxBodies][6];     // composite force, feet's wrenches subtracted
  double fiC[kMaxBodies][6];    // composite force of the bodies alone
  double M[kMaxBodies * kMaxBodies];  // mass matrix, then its Cholesky factor below the diagonal
  double Ld[kMaxBodies];        // the factor's diagonal
  double qdd[kMaxBodies];       // generalised force, then qdd0
  double z[kMaxCols];           // (x, u) of the stage
  double D[kMaxBodies][kMaxCols];  // d qdd / d(x, u), column per thread
  double pf[kMaxFeet][3];       // contact points, world
  uint32_t anc[kMaxBodies];     // ancestors of body i, itself included
  int bad;                      // 1 non-finite input, 2 mass matrix not positive definite
};

// One workgroup per (agent, stage): the derivatives of forward dynamics from
// those of inverse dynamics, d qdd / d x = -M^-1 d ID / d x at qdd = qdd0 and
// d qdd / d u = M^-1 d(S'tau + J'F) / d u, with d ID / d q and d ID / d qd in
// closed form from the tree's composite quantities: moving coordinate j moves
// its subtree rigidly along S_j, so each world-frame quantity of the subtree
// changes by S_j x (.), apart from terms through the parent's velocity and
// acceleration, which do not move, and the feet's world-fixed wrenches.
__global__ void __launch_bounds__(kLinThreads)
k_linearize(ModelDev md, int N, double dt, const double* __restrict__ X, const double* __restrict__ U,
            double* __restrict__ A, double* __restrict__ B, double* __restrict__ C,
            int32_t* __restrict__ status) {
  __shared__ LinLds L;
  const int tid = threadIdx.x;
  const int n = md.n, nx = 2 * n, nj = n - 6, nf = md.n_feet, fd = md.foot_dim;
  const int nu = nj + nf * fd, ncol = nx + nu;
  const int64_t ak = blockIdx.x;  // agent * N + stage
  const S6 a_root = s6(v3(0, 0, 0), v3(0, 0, md.gravity));
  const double* q = L.z;
  const double* qd = L.z + n;
  const double* F = L.z + nx + nj;

  if (tid == 0) L.bad = 0;
  __syncthreads();
  if (tid < ncol) {
    const double val = tid < nx ? X[ak * nx + tid] : U[ak * nu + tid - nx];
    L.z[tid] = val;
    if (!isfinite(val)) L.bad = 1;
  }
  if (tid < n) {
    uint32_t m = 1u << tid;
    for (int k = md.parent[tid]; k >= 0; k = md.parent[k]) m |= 1u << k;
    L.anc[tid] = m;
  }
  __syncthreads();
  if (L.bad) {
    if (tid == 0) atomicMax(status + ak / N, (int32_t)AGENT_NONFINITE);
    return;
  }
  // (1) world placement, motion subspace and inertia of body tid
  if (tid < n) {
    const int i = tid;
    M3 R;
    V3 p;
    joint_local(md, i, q[i], R, p);
    for (int k = md.parent[i]; k >= 0; k = md.parent[k]) {
      M3 Rk;
      V3 pk;
      joint_local(md, k, q[k], Rk, pk);
      p = pk + mul(Rk, p);
      R = mulM(Rk, R);
    }
    const V3 ax = mul(R, ld3(md.axis + 3 * i));
    st6(L.S[i], md.jtype[i] == 1 ? s6(v3(0, 0, 0), ax) : s6(ax, cross(p, ax)));
    const double m = md.mass[i];
    const V3 c = p + mul(R, ld3(md.com + 3 * i));
    const V3 J = ld3(md.inertia + 3 * i);
    double* I = L.Io[i];
    for (int u = 0; u < 3; ++u)
      for (int w = 0; w < 3; ++w) {
        // R diag(J) R' + m [c]x [c]x'
        double r = R.m[3 * u] * J.x * R.m[3 * w] + R.m[3 * u + 1] * J.y * R.m[3 * w + 1] +
                   R.m[3 * u + 2] * J.z * R.m[3 * w + 2];
        const double cu[3] = {c.x, c.y, c.z};
        r += m * ((u == w ? dot(c, c) : 0.0) - cu[u] * cu[w]);
        I[6 * u + w] = r;
        I[6 * (3 + u) + 3 + w] = u == w ? m : 0.0;
      }
    // m [c]x top right, its transpose bottom left
    const double cx[9] = {0, -c.z, c.y, c.z, 0, -c.x, -c.y, c.x, 0};
    for (int u = 0; u < 3; ++u)
      for (int w = 0; w < 3; ++w) {
        I[6 * u + 3 + w] = m * cx[3 * u + w];
        I[6 * (3 + u) + w] = m * cx[3 * w + u];
      }
    for (int f = 0; f < nf; ++f)
      if (md.foot_body[f] == i) {
        const V3 pt = p + mul(R, ld3(md.foot_offset + 3 * f));
        L.pf[f][0] = pt.x;
        L.pf[f][1] = pt.y;
        L.pf[f][2] = pt.z;
      }
  }
  __syncthreads();
  // (2) velocities
  if (tid < n) {
    S6 v = s6(v3(0, 0, 0), v3(0, 0, 0));
    for (int k = 0; k <= tid; ++k)
      if (L.anc[tid] >> k & 1u) v = v + qd[k] * ld6(L.S[k]);
    st6(L.v[tid], v);
  }
  __syncthreads();
  // (3) accelerations at qdd = 0, own forces, momenta and B = v x* I - I v x
  auto ext = [&](int i) {  // the feet's wrenches on body i
    S6 w = s6(v3(0, 0, 0), v3(0, 0, 0));
    for (int f = 0; f < nf; ++f)
      if (md.foot_body[f] == i) {
        const V3 force = ld3(F + f * fd);
        const V3 mom = fd == 6 ? ld3(F + f * fd + 3) : v3(0, 0, 0);
        w = w + s6(mom + cross(ld3(L.pf[f]), force), force);
      }
    return w;
  };
  if (tid < n) {
    const int i = tid;
    S6 a0 = a_root;
    for (int k = 0; k <= i; ++k)
      if (L.anc[i] >> k & 1u) a0 = a0 + qd[k] * crm(ld6(L.v[k]), ld6(L.S[k]));
    const S6 v = ld6(L.v[i]);
    const S6 h = mul6(L.Io[i], v);
    st6(L.a[i], a0);
    st6(L.hC[i], h);
    st6(L.fC[i], mul6(L.Io[i], a0) + crf(v, h) - ext(i));
    for (int c = 0; c < 6; ++c) {
      S6 e = s6(v3(0, 0, 0), v3(0, 0, 0));
      if (c < 3) (c == 0 ? e.a.x : c == 1 ? e.a.y : e.a.z) = 1.0;
      else (c == 3 ? e.b.x : c == 4 ? e.b.y : e.b.z) = 1.0;
      const S6 Ie = mul6(L.Io[i], e);
      const S6 col = crf(v, Ie) - mul6(L.Io[i], crm(v, e));
      const double cc[6] = {col.a.x, col.a.y, col.a.z, col.b.x, col.b.y, col.b.z};
      for (int r = 0; r < 6; ++r) L.BC[i][6 * r + c] = cc[r];
    }
    for (int e = 0; e < 36; ++e) L.IC[i][e] = L.Io[i][e];
  }
  __syncthreads();
  // (4) composites over subtrees (children come after their parents): one
  // thread per entry, bodies in reverse order
  if (tid < 84) {
    double* base;
    int stride, e;
    if (tid < 36) { base = &L.IC[0][0]; stride = 36; e = tid; }
    else if (tid < 72) { base = &L.BC[0][0]; stride = 36; e = tid - 36; }
    else if (tid < 78) { base = &L.hC[0][0]; stride = 6; e = tid - 72; }
    else { base = &L.fC[0][0]; stride = 6; e = tid - 78; }
    for (int i = n - 1; i > 0; --i) {
      const int par = md.parent[i];
      if (par >= 0) base[par * stride + e] += base[i * stride + e];
    }
  }
  __syncthreads();
  // (5) mass matrix M_ij = S_i' IC_j S_j (i an ancestor of j) and the
  // generalised force S'tau - ID(q, qd, 0, F)
  for (int idx = tid; idx < n * n; idx += kLinThreads) {
    const int i = idx / n, j = idx % n;
    double val = 0.0;
    if (L.anc[j] >> i & 1u) val = dot6(ld6(L.S[i]), mul6(L.IC[j], ld6(L.S[j])));
    else if (L.anc[i] >> j & 1u) val = dot6(ld6(L.S[j]), mul6(L.IC[i], ld6(L.S[i])));
    L.M[idx] = val;
  }
  if (tid < n) L.qdd[tid] = (tid >= 6 ? L.z[nx + tid - 6] : 0.0) - dot6(ld6(L.S[tid]), ld6(L.fC[tid]));
  __syncthreads();
  // (6) Cholesky factor, column by column (every thread forms the same pivot)
  for (int j = 0; j < n; ++j) {
    double d = L.M[j * n + j];
    for (int t = 0; t < j; ++t) d -= L.M[j * n + t] * L.M[j * n + t];
    if (!(d > 0.0)) {
      if (tid == 0) atomicMax(status + ak / N, (int32_t)AGENT_NOT_PD);
      return;
    }
    const double l = sqrt(d);
    const int i = j + 1 + tid;
    if (i < n) {
      double s = L.M[i * n + j];
      for (int t = 0; t < j; ++t) s -= L.M[i * n + t] * L.M[j * n + t];
      L.M[i * n + j] = s / l;
    }
    if (tid == 0) L.Ld[j] = l;
    __syncthreads();
  }
  // (7) qdd0 = M^-1 (S'tau + J'F - h)
  if (tid == 0) {
    for (int i = 0; i < n; ++i) {
      double s = L.qdd[i];
      for (int t = 0; t < i; ++t) s -= L.M[i * n + t] * L.qdd[t];
      L.qdd[i] = s / L.Ld[i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = L.qdd[i];
      for (int t = i + 1; t < n; ++t) s -= L.M[t * n + i] * L.qdd[t];
      L.qdd[i] = s / L.Ld[i];
    }
  }
  __syncthreads();
  // (8) accelerations and forces at qdd0
  if (tid < n) {
    const int i = tid;
    S6 a = ld6(L.a[i]);
    for (int k = 0; k <= i; ++k)
      if (L.anc[i] >> k & 1u) a = a + L.qdd[k] * ld6(L.S[k]);
    st6(L.a[i], a);
    const S6 v = ld6(L.v[i]);
    const S6 fi = mul6(L.Io[i], a) + crf(v, mul6(L.Io[i], v));
    st6(L.fiC[i], fi);
    st6(L.fC[i], fi - ext(i));
  }
  __syncthreads();
  if (tid < 12) {
    double* base = tid < 6 ? &L.fiC[0][0] : &L.fC[0][0];
    const int e = tid % 6;
    for (int i = n - 1; i > 0; --i) {
      const int par = md.parent[i];
      if (par >= 0) base[par * 6 + e] += base[i * 6 + e];
    }
  }
  __syncthreads();
  // (9) one column of d qdd / d(x, u) per thread
  if (tid < ncol) {
    const int t = tid;
    if (t < nx) {
      const int j = t % n;
      const S6 Sj = ld6(L.S[j]);
      const int par = md.parent[j];
      const S6 vp = par >= 0 ? ld6(L.v[par]) : s6(v3(0, 0, 0), v3(0, 0, 0));
      if (t < n) {
        // d ID / d q_j
        const S6 ap = par >= 0 ? ld6(L.a[par]) : a_root;
        const S6 dv = crm(Sj, vp);
        const S6 al = crm(Sj, ap) - crm(dv, vp);
        auto psi = [&](int i) {
          S6 r = crf(Sj, ld6(L.fiC[i])) - mul6(L.IC[i], al) - mul6(L.BC[i], dv) - crf(dv, ld6(L.hC[i]));
          for (int f = 0; f < nf; ++f) {
            const int b = md.foot_body[f];
            if (L.anc[b] >> i & 1u) {  // foot in the subtree of i
              const V3 pt = ld3(L.pf[f]);
              r.a = r.a - cross(Sj.b + cross(Sj.a, pt), ld3(F + f * fd));
            }
          }
          return r;
        };
        const S6 psij = psi(j);
        for (int i = 0; i < n; ++i) {
          double d = 0.0;
          const S6 Si = ld6(L.S[i]);
          if (L.anc[i] >> j & 1u) d = dot6(crm(Sj, Si), ld6(L.fC[i])) + dot6(Si, i == j ? psij : psi(i));
          else if (L.anc[j] >> i & 1u) d = dot6(Si, psij);
          L.D[i][t] = -d;
        }
      } else {
        // d ID / d qd_j
        const S6 w = crm(Sj, vp);
        auto phi = [&](int i) {
          return mul6(L.BC[i], Sj) + crf(Sj, ld6(L.hC[i])) - 2.0 * mul6(L.IC[i], w);
        };
        const S6 phij = phi(j);
        for (int i = 0; i < n; ++i) {
          double d = 0.0;
          const S6 Si = ld6(L.S[i]);
          if (L.anc[i] >> j & 1u) d = dot6(Si, i == j ? phij : phi(i));
          else if (L.anc[j] >> i & 1u) d = dot6(Si, phij);
          L.D[i][t] = -d;
        }
      }
    } else if (t < nx + nj) {
      for (int i = 0; i < n; ++i) L.D[i][t] = i == 6 + (t - nx) ? 1.0 : 0.0;
    } else {
      const int w = t - nx - nj, f = w / fd, comp = w % fd;
      S6 e = s6(v3(0, 0, 0), v3(0, 0, 0));
      V3 unit = v3(comp % 3 == 0, comp % 3 == 1, comp % 3 == 2);
      if (comp < 3) e = s6(cross(ld3(L.pf[f]), unit), unit);
      else e = s6(unit, v3(0, 0, 0));
      const uint32_t up = L.anc[md.foot_body[f]];
      for (int i = 0; i < n; ++i) L.D[i][t] = (up >> i & 1u) ? dot6(ld6(L.S[i]), e) : 0.0;
    }
    // M^-1 on the column
    for (int i = 0; i < n; ++i) {
      double s = L.D[i][t];
      for (int k = 0; k < i; ++k) s -= L.M[i * n + k] * L.D[k][t];
      L.D[i][t] = s / L.Ld[i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = L.D[i][t];
      for (int k = i + 1; k < n; ++k) s -= L.M[k * n + i] * L.D[k][t];
      L.D[i][t] = s / L.Ld[i];
    }
    // q+ = q + dt qd + dt^2 qdd, qd+ = qd + dt qdd
    const double dt2 = dt * dt;
    if (t < nx) {
      double* Ak = A + ak * nx * nx;
      for (int r = 0; r < n; ++r) {
        const double dq = L.D[r][t];
        Ak[r * nx + t] = (r == t ? 1.0 : 0.0) + (r + n == t ? dt : 0.0) + dt2 * dq;
        Ak[(n + r) * nx + t] = (r + n == t ? 1.0 : 0.0) + dt * dq;
      }
    } else {
      double* Bk = B + ak * nx * nu;
      const int c = t - nx;
      for (int r = 0; r < n; ++r) {
        Bk[r * nu + c] = dt2 * L.D[r][t];
        Bk[(n + r) * nu + c] = dt * L.D[r][t];
      }
    }
  }
  __syncthreads();
  // (10) c = f(x, u) - A x - B u = (dt^2 r, dt r), r = qdd0 - D (x, u)
  if (tid < n) {
    double r = L.qdd[tid];
    for (int t = 0; t < ncol; ++t) r -= L.D[tid][t] * L.z[t];
    C[ak * nx + tid] = dt * dt * r;
    C[ak * nx + n + tid] = dt * r;
  }
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
  const int64_t blocks = (int64_t)n_agents * N;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_linearize, dim3((unsigned)blocks), dim3(kLinThreads), 0, s, md, N, dt, X, U, A, B,
                     C, status);
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
