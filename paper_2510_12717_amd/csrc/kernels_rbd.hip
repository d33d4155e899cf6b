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
    tau[i] = (md.jtype[i] == 1 ? dot(ax, ff[i]) : dot(ax, fn[i])) + md.armature[i] * qdd[i];
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

// Lane `lane`'s value of v (lane a compile-time or wave-uniform index).
__device__ inline double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffu), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
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
// Row stride of a 6x6 spatial inertia in LDS: 37 doubles, so that the lanes of
// a per-body phase (lane i on body i) fall on different banks (a stride of 36
// doubles put every fourth body on the same banks; padding the 6-double
// spatial vectors to 7 as well measured no further gain).
constexpr int kIS = 37;

struct LinLds {
  double S[kMaxBodies][6];      // joint motion subspace
  double v[kMaxBodies][6];      // velocity
  double a[kMaxBodies][6];      // acceleration: qdd = 0 first, then qdd = qdd0
  // arrays whose lifetimes do not overlap share storage
  union {
    double Io[kMaxBodies][kIS];  // own spatial inertia (until the forces at qdd0)
    struct {
      double dv[kMaxBodies][6];   // S_j x v_parent(j)
      double al[kMaxBodies][6];   // S_j x a_parent(j) - dv_j x v_parent(j)
      double psi[kMaxBodies][6];  // d(composite force of j's subtree)/d q_j
      double phi[kMaxBodies][6];  // d(composite force of j's subtree)/d qd_j
    };
  };
  union {
    struct {
      double Rl[kMaxBodies][9];   // body's rotation relative to its parent (placement only)
      double pl[kMaxBodies][3];   // body's origin in the parent frame (placement only)
    };
    struct {
      double IC[kMaxBodies][kIS];  // composite inertia of the subtree
      double BC[kMaxBodies][kIS];  // composite of v x* I - I v x
      double fC[kMaxBodies][6];   // composite force, feet's wrenches subtracted
      double fiC[kMaxBodies][6];  // composite force of the bodies alone
    };
    double D[kMaxBodies][kMaxCols];  // d qdd / d(x, u), column per thread (columns phase on)
  };
  double hC[kMaxBodies][6];     // composite momentum
  double Fv[kMaxBodies][6];     // IC_i S_i
  double G[kMaxBodies][6];      // BC_i' S_i
  double eC[kMaxBodies][6];     // the feet's wrenches on i's subtree (fiC - fC)
  double PF[kMaxBodies][9];     // sum over the feet below i of p_f F_f'
  double sF[kMaxBodies];        // sum over the feet below i of p_f . F_f
  // mass matrix, then its Cholesky factor on and below the diagonal, row
  // stride kMaxBodies, rows and columns past n padded with the identity
  double M[kMaxBodies * kMaxBodies];
  double iLd[kMaxBodies];       // reciprocals of the factor's diagonal
  double qdd[kMaxBodies];       // generalised force, then qdd0
  double z[kMaxCols];           // (x, u) of the stage
  double pf[kMaxFeet][3];       // contact points, world
  uint32_t anc[kMaxBodies];     // ancestors of body i, itself included
  int bad;                      // 1 non-finite input, 2 mass matrix not positive definite
};
static_assert(sizeof(LinLds) <= 40 * 1024, "four workgroups per CU");

// One workgroup per (agent, stage): the derivatives of forward dynamics from
// those of inverse dynamics, d qdd / d x = -M^-1 d ID / d x at qdd = qdd0 and
// d qdd / d u = M^-1 d(S'tau + J'F) / d u, with d ID / d q and d ID / d qd in
// closed form from the tree's composite quantities: moving coordinate j moves
// its subtree rigidly along S_j, so each world-frame quantity of the subtree
// changes by S_j x (.), apart from terms through the parent's velocity and
// acceleration, which do not move, and the feet's world-fixed wrenches.
template <typename T>
__global__ void __launch_bounds__(kLinThreads)
k_linearize(ModelDev md, int N, double dt, const T* __restrict__ X, const T* __restrict__ U,
            T* __restrict__ A, T* __restrict__ B, T* __restrict__ C, T* __restrict__ Jf,
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
    // x of the stage in the solution layout (N + 1 states per agent)
    const double val = tid < nx ? (double)X[(ak + ak / N) * nx + tid] : (double)U[ak * nu + tid - nx];
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
  // (1) world placement, motion subspace and inertia of body tid (each body's
  // placement relative to its parent first, then composed up the chain)
  if (tid < n) {
    M3 R;
    V3 p;
    joint_local(md, tid, q[tid], R, p);
    for (int k = 0; k < 9; ++k) L.Rl[tid][k] = R.m[k];
    L.pl[tid][0] = p.x;
    L.pl[tid][1] = p.y;
    L.pl[tid][2] = p.z;
  }
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    M3 R;
    for (int k = 0; k < 9; ++k) R.m[k] = L.Rl[i][k];
    V3 p = ld3(L.pl[i]);
    for (int k = md.parent[i]; k >= 0; k = md.parent[k]) {
      M3 Rk;
      for (int e = 0; e < 9; ++e) Rk.m[e] = L.Rl[k][e];
      p = ld3(L.pl[k]) + mul(Rk, p);
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
  // the feet's no-slip rows J_f v = 0 at the stage-0 configuration: zero on
  // the positions; on the velocities the contact point's linear velocity and
  // (6D feet) the foot's angular velocity per unit qd_i, i an ancestor of the foot
  if (Jf && ak % N == 0) {
    const int nfd = nf * fd;
    T* Jo = Jf + (ak / N) * (int64_t)nfd * nx;
    for (int idx = tid; idx < nfd * nx; idx += kLinThreads) {
      const int row = idx / nx, col = idx % nx, f = row / fd, comp = row % fd;
      double v = 0.0;
      if (col >= n && (L.anc[md.foot_body[f]] >> (col - n) & 1u)) {
        const S6 Si = ld6(L.S[col - n]);
        const V3 sel = comp < 3 ? Si.b + cross(Si.a, ld3(L.pf[f])) : Si.a;
        const int c3 = comp % 3;
        v = c3 == 0 ? sel.x : c3 == 1 ? sel.y : sel.z;
      }
      Jo[idx] = (T)v;
    }
  }
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
    double I[36];  // the body's inertia, in registers for this phase
#pragma unroll
    for (int e = 0; e < 36; ++e) I[e] = L.Io[i][e];
    const S6 h = mul6(I, v);
    st6(L.a[i], a0);
    st6(L.hC[i], h);
    st6(L.fC[i], mul6(I, a0) + crf(v, h) - ext(i));
    // B e_c = v x* (I e_c) - I (v x e_c), column by column
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const S6 Ie = s6(v3(I[c], I[6 + c], I[12 + c]), v3(I[18 + c], I[24 + c], I[30 + c]));
      S6 e = s6(v3(0, 0, 0), v3(0, 0, 0));
      if (c < 3) (c == 0 ? e.a.x : c == 1 ? e.a.y : e.a.z) = 1.0;
      else (c == 3 ? e.b.x : c == 4 ? e.b.y : e.b.z) = 1.0;
      const S6 col = crf(v, Ie) - mul6(I, crm(v, e));
      L.BC[i][c] = col.a.x;
      L.BC[i][6 + c] = col.a.y;
      L.BC[i][12 + c] = col.a.z;
      L.BC[i][18 + c] = col.b.x;
      L.BC[i][24 + c] = col.b.y;
      L.BC[i][30 + c] = col.b.z;
    }
#pragma unroll
    for (int e = 0; e < 36; ++e) L.IC[i][e] = I[e];
  }
  __syncthreads();
  // (4) composites over subtrees (children come after their parents): one
  // thread per entry, bodies in reverse order
  if (tid < 84) {
    double* base;
    int stride, e;
    if (tid < 36) { base = &L.IC[0][0]; stride = kIS; e = tid; }
    else if (tid < 72) { base = &L.BC[0][0]; stride = kIS; e = tid - 36; }
    else if (tid < 78) { base = &L.hC[0][0]; stride = 6; e = tid - 72; }
    else { base = &L.fC[0][0]; stride = 6; e = tid - 78; }
    for (int i = n - 1; i > 0; --i) {
      const int par = md.parent[i];
      if (par >= 0) base[par * stride + e] += base[i * stride + e];
    }
  }
  __syncthreads();
  // (5) per-body IC_i S_i and BC_i' S_i; the generalised force
  // S'tau - ID(q, qd, 0, F)
  if (tid < n) {
    const int i = tid;
    const S6 Si = ld6(L.S[i]);
    st6(L.Fv[i], mul6(L.IC[i], Si));
    double g[6];
    const double sv[6] = {Si.a.x, Si.a.y, Si.a.z, Si.b.x, Si.b.y, Si.b.z};
    for (int c = 0; c < 6; ++c) {
      double t = 0.0;
      for (int r = 0; r < 6; ++r) t += L.BC[i][6 * r + c] * sv[r];
      g[c] = t;
    }
    for (int c = 0; c < 6; ++c) L.G[i][c] = g[c];
    L.qdd[i] = (i >= 6 ? L.z[nx + i - 6] : 0.0) - dot6(Si, ld6(L.fC[i]));
  } else if (tid < kMaxBodies) {
    L.qdd[tid] = 0.0;
  }
  __syncthreads();
  // (6) mass matrix M_ij = S_i' IC_j S_j (i an ancestor of j), padded
  for (int idx = tid; idx < kMaxBodies * kMaxBodies; idx += kLinThreads) {
    const int i = idx / kMaxBodies, j = idx % kMaxBodies;
    double val = i == j ? 1.0 : 0.0;
    if (i < n && j < n) {
      if (i == j) val = dot6(ld6(L.S[i]), ld6(L.Fv[i])) + md.armature[i];
      else if (L.anc[j] >> i & 1u) val = dot6(ld6(L.S[i]), ld6(L.Fv[j]));
      else if (L.anc[i] >> j & 1u) val = dot6(ld6(L.S[j]), ld6(L.Fv[i]));
      else val = 0.0;
    }
    L.M[idx] = val;
  }
  __syncthreads();
  // (7) wavefront 0: Cholesky factor with lane i holding row i in registers
  // (pivots and multipliers broadcast with readlane), then the forward sweep
  // of qdd0; the transposed sweep after the factor is in LDS
  if (tid < 64) {
    const int i = tid;
    double r[kMaxBodies];
#pragma unroll
    for (int k = 0; k < kMaxBodies; ++k) r[k] = i < kMaxBodies ? L.M[i * kMaxBodies + k] : 0.0;
    bool ok = true;
    double inv_own = 1.0;  // reciprocal of this lane's pivot
#pragma unroll
    for (int j = 0; j < kMaxBodies; ++j) {
      const double d = readlane_d(r[j], j);
      ok = ok && d > 0.0;
      const double l = sqrt(d), inv = 1.0 / l;
      r[j] = i == j ? l : r[j] * inv;
      inv_own = i == j ? inv : inv_own;
#pragma unroll
      for (int k = j + 1; k < kMaxBodies; ++k) r[k] -= r[j] * readlane_d(r[j], k);
    }
    if (!ok) {
      if (i == 0) atomicMax(status + ak / N, (int32_t)AGENT_NOT_PD);
    } else if (i < kMaxBodies) {
#pragma unroll
      for (int k = 0; k < kMaxBodies; ++k)
        if (k <= i) L.M[i * kMaxBodies + k] = r[k];
      L.iLd[i] = inv_own;
    }
    double g = i < kMaxBodies ? L.qdd[i] : 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBodies; ++k) {
      const double yk = readlane_d(g, k) * readlane_d(inv_own, k);
      g = i == k ? yk : (i > k ? g - r[k] * yk : g);
    }
    if (i < kMaxBodies) L.qdd[i] = g;
    if (i == 0) L.bad = ok ? 0 : 2;
  }
  __syncthreads();
  if (L.bad) return;
  if (tid < 64) {
    const int i = tid;
    double g = i < kMaxBodies ? L.qdd[i] : 0.0;
#pragma unroll
    for (int k = kMaxBodies - 1; k >= 0; --k) {
      const double xk = readlane_d(g, k) * L.iLd[k];
      const double lki = i < k ? L.M[k * kMaxBodies + i] : 0.0;
      g = i == k ? xk : g - lki * xk;
    }
    if (i < kMaxBodies) L.qdd[i] = g;
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
    double I[36];
#pragma unroll
    for (int e = 0; e < 36; ++e) I[e] = L.Io[i][e];
    const S6 fi = mul6(I, a) + crf(v, mul6(I, v));
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
  // (9) per coordinate j (wavefront 0: q_j, wavefront 1: qd_j): the change of
  // the composite force of j's subtree.  Moving q_j moves the subtree rigidly
  // along S_j except for the parent's velocity and acceleration and the feet's
  // world-fixed wrenches; qd_j enters the subtree's velocities as S_j.
  if ((tid & 63) < n) {
    const int j = tid & 63;
    const S6 Sj = ld6(L.S[j]);
    const int par = md.parent[j];
    const S6 vp = par >= 0 ? ld6(L.v[par]) : s6(v3(0, 0, 0), v3(0, 0, 0));
    const S6 dvj = crm(Sj, vp);
    if (tid < 64) {
      const S6 ap = par >= 0 ? ld6(L.a[par]) : a_root;
      const S6 alj = crm(Sj, ap) - crm(dvj, vp);
      S6 ps = crf(Sj, ld6(L.fiC[j])) - mul6(L.IC[j], alj) - mul6(L.BC[j], dvj) - crf(dvj, ld6(L.hC[j]));
      for (int f = 0; f < nf; ++f)
        if (L.anc[md.foot_body[f]] >> j & 1u)
          ps.a = ps.a - cross(Sj.b + cross(Sj.a, ld3(L.pf[f])), ld3(F + f * fd));
      st6(L.dv[j], dvj);
      st6(L.al[j], alj);
      st6(L.psi[j], ps);
    } else {
      st6(L.phi[j], mul6(L.BC[j], Sj) + crf(Sj, ld6(L.hC[j])) - 2.0 * mul6(L.IC[j], dvj));
      st6(L.eC[j], ld6(L.fiC[j]) - ld6(L.fC[j]));
      double P[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, sp = 0.0;
      for (int f = 0; f < nf; ++f)
        if (L.anc[md.foot_body[f]] >> j & 1u) {
          const V3 pt = ld3(L.pf[f]), fo = ld3(F + f * fd);
          const double pa[3] = {pt.x, pt.y, pt.z}, fa[3] = {fo.x, fo.y, fo.z};
#pragma unroll
          for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int w = 0; w < 3; ++w) P[3 * u + w] += pa[u] * fa[w];
          sp += dot(pt, fo);
        }
#pragma unroll
      for (int e = 0; e < 9; ++e) L.PF[j][e] = P[e];
      L.sF[j] = sp;
    }
  }
  __syncthreads();
  // (10) columns of d qdd / d(x, u): wavefront 0 takes the q columns and the
  // joint torques, wavefront 1 the qd columns and the foot wrenches, one per
  // lane.  For body i in the subtree of coordinate j the derivative of ID_i
  // reduces to products with the per-body vectors IC_i S_i and BC_i' S_i; for
  // an ancestor i of j it is S_i' times the composite change at j.
  const int wave = tid >> 6, lane = tid & 63;
  const int nw = nf * fd;
  const int t = wave == 0 ? (lane < n ? lane : (lane < n + nj ? nx + lane - n : -1))
                          : (lane < n ? n + lane : (lane < n + nw ? nx + nj + lane - n : -1));
  if (t >= 0) {
    if (t < nx) {
      const int j = t % n;
      const S6 Sj = ld6(L.S[j]);
      const S6 dv = ld6(L.dv[j]);
      if (t < n) {
        // d ID / d q_j
        const S6 al = ld6(L.al[j]);
        const S6 psij = ld6(L.psi[j]);
        for (int i = 0; i < n; ++i) {
          double d = 0.0;
          const S6 Si = ld6(L.S[i]);
          if (L.anc[i] >> j & 1u) {
            // the feet below body i: sum of (velocity of the contact point
            // under S_j) x force = S_j.lin x F_sum + PF S_j.ang - S_j.ang sF
            const S6 eC = ld6(L.eC[i]);
            const double* P = L.PF[i];
            const V3 PS = v3(P[0] * Sj.a.x + P[1] * Sj.a.y + P[2] * Sj.a.z,
                             P[3] * Sj.a.x + P[4] * Sj.a.y + P[5] * Sj.a.z,
                             P[6] * Sj.a.x + P[7] * Sj.a.y + P[8] * Sj.a.z);
            const V3 ft = cross(Sj.b, eC.b) + PS - L.sF[i] * Sj.a;
            d = -dot6(crm(Sj, Si), eC) - dot6(al, ld6(L.Fv[i])) - dot6(dv, ld6(L.G[i])) +
                dot6(crm(dv, Si), ld6(L.hC[i])) - dot(Si.a, ft);
          } else if (L.anc[j] >> i & 1u) {
            d = dot6(Si, psij);
          }
          L.D[i][t] = -d;
        }
      } else {
        // d ID / d qd_j
        const S6 phij = ld6(L.phi[j]);
        for (int i = 0; i < n; ++i) {
          double d = 0.0;
          const S6 Si = ld6(L.S[i]);
          if (L.anc[i] >> j & 1u)
            d = dot6(Sj, ld6(L.G[i])) - dot6(crm(Sj, Si), ld6(L.hC[i])) - 2.0 * dot6(dv, ld6(L.Fv[i]));
          else if (L.anc[j] >> i & 1u)
            d = dot6(Si, phij);
          L.D[i][t] = -d;
        }
      }
    } else if (t < nx + nj) {
      for (int i = 0; i < n; ++i) L.D[i][t] = i == 6 + (t - nx) ? 1.0 : 0.0;
    } else {
      const int wi = t - nx - nj, f = wi / fd, comp = wi % fd;
      const V3 unit = v3(comp % 3 == 0, comp % 3 == 1, comp % 3 == 2);
      const S6 e = comp < 3 ? s6(cross(ld3(L.pf[f]), unit), unit) : s6(unit, v3(0, 0, 0));
      const uint32_t up = L.anc[md.foot_body[f]];
      for (int i = 0; i < n; ++i) L.D[i][t] = (up >> i & 1u) ? dot6(ld6(L.S[i]), e) : 0.0;
    }
    // M^-1 on the column, in registers (rows past n: identity)
    double y[kMaxBodies];
#pragma unroll
    for (int i = 0; i < kMaxBodies; ++i) y[i] = i < n ? L.D[i][t] : 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBodies; ++k) {
      y[k] *= L.iLd[k];
#pragma unroll
      for (int i = k + 1; i < kMaxBodies; ++i) y[i] -= L.M[i * kMaxBodies + k] * y[k];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = kMaxBodies - 1; k >= 0; --k) {
      y[k] *= L.iLd[k];
#pragma unroll
      for (int i = 0; i < k; ++i) y[i] -= L.M[k * kMaxBodies + i] * y[k];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < kMaxBodies; ++r)
      if (r < n) L.D[r][t] = y[r];
  }
  __syncthreads();
  // (11) A and B column by column (q+ = q + dt qd + dt^2 qdd, qd+ = qd + dt
  // qdd), after the barrier so that it waits on no global store
  if (t >= 0) {
    const double dt2 = dt * dt;
    for (int r = 0; r < n; ++r) {
      const double yr = L.D[r][t];
      if (t < nx) {
        T* Ak = A + ak * nx * nx;
        Ak[r * nx + t] = (T)((r == t ? 1.0 : 0.0) + (r + n == t ? dt : 0.0) + dt2 * yr);
        Ak[(n + r) * nx + t] = (T)((r + n == t ? 1.0 : 0.0) + dt * yr);
      } else {
        T* Bk = B + ak * nx * nu;
        Bk[r * nu + t - nx] = (T)(dt2 * yr);
        Bk[(n + r) * nu + t - nx] = (T)(dt * yr);
      }
    }
  }
  // (12) c = f(x, u) - A x - B u = (dt^2 r, dt r), r = qdd0 - D (x, u)
  if (tid < n) {
    double r = L.qdd[tid];
    for (int t = 0; t < ncol; ++t) r -= L.D[tid][t] * L.z[t];
    C[ak * nx + tid] = (T)(dt * dt * r);
    C[ak * nx + n + tid] = (T)(dt * r);
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

// Thread per agent; x [count][N + 1][nx] and u [count][N][nu] in the solution
// layout (x_0, x_1 and u_0 used), measured state xm [count][nx], tau [count][nj].
template <typename T>
__global__ void __launch_bounds__(64)
k_rti_torque(ModelDev md, int count, int N, double dt, double kp, double kd, const T* __restrict__ X,
             const T* __restrict__ U, const T* __restrict__ xm, T* __restrict__ tau) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int n = md.n, nx = 2 * n, nj = n - 6, nf = md.n_feet * md.foot_dim, nu = nj + nf;
  const T* x = X + (int64_t)t * (N + 1) * nx;
  const T* u = U + (int64_t)t * N * nu;
  double x0[2 * kMaxBodies], qdd[kMaxBodies], F[kMaxU], tr[kMaxBodies];
  for (int i = 0; i < nx; ++i) x0[i] = (double)x[i];
  for (int i = 0; i < n; ++i) qdd[i] = ((double)x[nx + n + i] - x0[n + i]) / dt;
  for (int i = 0; i < nf; ++i) F[i] = (double)u[nj + i];
  rnea_dev(md, x0, x0 + n, qdd, F, tr);
  for (int i = 0; i < nj; ++i)
    tau[(int64_t)t * nj + i] = (T)(kp * (x0[6 + i] - (double)xm[(int64_t)t * nx + 6 + i]) +
                                   kd * (x0[n + 6 + i] - (double)xm[(int64_t)t * nx + n + 6 + i]) +
                                   tr[6 + i]);
}

}  // namespace

hipError_t launch_rnea(const ModelDev& md, int count, const double* q, const double* qd,
                       const double* qdd, const double* F, double* tau, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rnea, dim3((count + 63) / 64), dim3(64), 0, s, md, count, q, qd, qdd, F, tau);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_linearize(const ModelDev& md, int n_agents, int N, double dt, const T* X, const T* U,
                            T* A, T* B, T* C, T* Jf, int32_t* status, hipStream_t s) {
  const int64_t blocks = (int64_t)n_agents * N;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_linearize<T>, dim3((unsigned)blocks), dim3(kLinThreads), 0, s, md, N, dt, X, U, A,
                     B, C, Jf, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rti_torque(const ModelDev& md, int count, int N, double dt, double kp, double kd,
                             const T* X, const T* U, const T* xm, T* tau, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rti_torque<T>, dim3((count + 63) / 64), dim3(64), 0, s, md, count, N, dt, kp, kd,
                     X, U, xm, tau);
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
  for (int i = 0; i < n; ++i) {
    const double a = d->armature ? d->armature[i] : 0.0;
    if (!(std::isfinite(a) && a >= 0.0))
      return api_fail(MPC_ERR_INVALID_ARG, "model: armature must be finite and non-negative");
  }
  MPC_HIP_TRY(hipSetDevice(device));
  const size_t dbl = (size_t)n * (3 + 3 + 1 + 3 + 3 + 1) + (size_t)nf * 3;
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
               oc = putd(d->com, 3 * n), oi = putd(d->inertia, 3 * n);
  const size_t oar = o;
  for (int i = 0; i < n; ++i) hd[o + i] = d->armature ? d->armature[i] : 0.0;
  o += n;
  const size_t of = nf ? putd(d->foot_offset, 3 * nf) : o;
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
                   dd + oar, nf ? di + 2 * n : nullptr, nf ? dd + of : nullptr};
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
                                    int32_t precision, const void* x, const void* u, void* A, void* B,
                                    void* c, void* J_foot, int32_t* status, void* stream) {
  using namespace mpc;
  if (!m || n_agents < 0 || N < 1 || N > 64 || !(dt > 0))
    return api_fail(MPC_ERR_INVALID_ARG, "n_agents >= 0, 1 <= N <= 64 and dt > 0 required");
  if (precision != MPC_FP64 && precision != MPC_FP32)
    return api_fail(MPC_ERR_INVALID_ARG, "precision: MPC_FP64 (double io) or MPC_FP32 (float io)");
  if (n_agents > 0 && (!x || !u || !A || !B || !c || !status))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument");
  MPC_HIP_TRY(hipSetDevice(m->device));
  const hipStream_t s = (hipStream_t)stream;
  if (precision == MPC_FP64)
    MPC_HIP_TRY(launch_linearize(m->md, n_agents, N, dt, (const double*)x, (const double*)u, (double*)A,
                                 (double*)B, (double*)c, (double*)J_foot, status, s));
  else
    MPC_HIP_TRY(launch_linearize(m->md, n_agents, N, dt, (const float*)x, (const float*)u, (float*)A,
                                 (float*)B, (float*)c, (float*)J_foot, status, s));
  return MPC_OK;
}

extern "C" mpc_status mpc_rti_torque(mpc_model_t m, int32_t count, int32_t N, double dt, double kp,
                                     double kd, int32_t precision, const void* x, const void* u,
                                     const void* x_meas, void* tau, void* stream) {
  using namespace mpc;
  if (!m || count < 0 || N < 1 || N > 64 || !(dt > 0) || (count > 0 && (!x || !u || !x_meas || !tau)))
    return api_fail(MPC_ERR_INVALID_ARG, "null argument, N outside 1..64, or dt <= 0");
  if (precision != MPC_FP64 && precision != MPC_FP32)
    return api_fail(MPC_ERR_INVALID_ARG, "precision: MPC_FP64 (double io) or MPC_FP32 (float io)");
  MPC_HIP_TRY(hipSetDevice(m->device));
  const hipStream_t s = (hipStream_t)stream;
  if (precision == MPC_FP64)
    MPC_HIP_TRY(launch_rti_torque(m->md, count, N, dt, kp, kd, (const double*)x, (const double*)u,
                                  (const double*)x_meas, (double*)tau, s));
  else
    MPC_HIP_TRY(launch_rti_torque(m->md, count, N, dt, kp, kd, (const float*)x, (const float*)u,
                                  (const float*)x_meas, (float*)tau, s));
  return MPC_OK;
}
