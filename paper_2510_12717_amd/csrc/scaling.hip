// Alg. 1's scaling step (f_Ruiz: Ruiz equilibration of the KKT system before
// the factorisation) and the residual-balancing rho update of the OSQP
// iteration the paper adopts (Sec. III-B), on the device.
//
// k_ruiz runs the equilibration of one agent per workgroup on the stacked
// KKT matrix [[P, A'], [A, 0]] (primal x_1..x_N, u_0..u_{N-1}; rows: the
// dynamics x_{k+1} - A_k x_k - B_k u_k and the constraint rows C_k u_k):
// every round divides each primal column and each dynamics row by the square
// root of its infinity norm (norms below 1e-4 count as 1, above 1e4 as 1e4)
// and then the cost by max(mean column norm of P, |q|_inf).  The scales are
// tied so that the scaled problem has the solver's form: a state or input
// component has one scale over the stages, f_x and f_y of every foot share
// one scale and each other force or moment component one scale over the
// feet, and a constraint row's scale follows from its inputs' (1/d_j on
// identity rows, 1/d_fxy on the pyramid facets, whose friction coefficient
// becomes mu d_fz / d_fxy).  It then writes the scaled problem data next to
// the caller's (D^-1 A_k D, D^-1 B_k D_u, D^-1 c_k, c D Q D, c D_u R D_u,
// D^-1 x_ref, D^-1 x0, tau_max / d_tau) and moves a warm start into the
// scaled variables (u / d_u, E z, c y / E).  The dynamics-row scales only
// shape the column norms: the iteration keeps the dynamics exact.
//
// k_unscale maps the iterate back (x = D x^, u = D_u u^, z = z^ / E,
// y = E y^ / c).  k_rho_update forms OSQP's estimate
// rho sqrt((|r_prim| / max(|Cu|, |z|)) / (|r_dual| / max(|Px|, |C'y|, |q|)))
// from the residual kernel's primal and dual residuals of the scaled problem,
// clips it to [1e-6, 1e6], rounds it to a power of 2^(1/4), and adopts it
// when it moved rho by more than the tolerance either way.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mpc_internal.h"
#include "scaling.h"
#include "stage_rows.h"

namespace mpc {
namespace {

constexpr double kNormFloor = 1e-4, kNormCeil = 1e4;
constexpr double kRhoLo = 1e-6, kRhoHi = 1e6;
constexpr int kThreads = 256;
constexpr int kMaxNx = 64, kMaxNu = 32;

__device__ inline double clamp_norm(double v) { return v < kNormFloor ? 1.0 : fmin(v, kNormCeil); }

// Tied scale of input j: torques their own, foot components one per
// component over the feet with f_y on f_x's.
__device__ inline int tie_of(const AgentDesc& d, int j) {
  if (j < d.n_tau) return j;
  const int c = (j - d.n_tau) % d.foot_dim;
  return d.n_tau + (c == 1 ? 0 : c);
}

// Scale of constraint row i (identity rows 1/d_i, facets of a foot 1/d_fx).
__device__ inline double row_scale(const AgentDesc& d, int i, const double* Du) {
  if (i < d.nu) return 1.0 / Du[i];
  const int f = (i - d.nu) >> 2;
  return 1.0 / Du[d.n_tau + f * d.foot_dim];
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_ruiz(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
       Inputs<T> in, int rounds, ScaledInputs<T> out, double* __restrict__ scale, int warm,
       State<T> st) {
  const int agent = list ? list[blockIdx.x] : (int)blockIdx.x;
  const AgentDesc d = desc[agent];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m, tid = threadIdx.x, nt = blockDim.x;
  __shared__ double Dx[kMaxNx], Du[kMaxNu], Ed[kMaxNx];
  __shared__ double colx[kMaxNx], colu[kMaxNu], rowd[kMaxNx], cpart[kThreads / 64], cmax[kThreads / 64];
  __shared__ double cs;
  __shared__ T sA[kMaxNx * kMaxNx], sB[kMaxNx * kMaxNu];  // one stage's A_k and B_k
  const T* q = in.q + d.oq;
  const T* r = in.r + d.orr;
  const T* xr = in.xr + d.oxr;
  const double mu = (double)in.mu[d.omu];
  for (int j = tid; j < nx; j += nt) {
    Dx[j] = 1.0;
    Ed[j] = 1.0;
  }
  for (int j = tid; j < nu; j += nt) Du[j] = 1.0;
  if (tid == 0) cs = 1.0;
  __syncthreads();
  for (int it = 0; it < rounds; ++it) {
    // column norms of x (P, the identity of the row x_k enters, A_k of the next
    // row), of u (P, B_k, constraint rows), row norms of the dynamics
    for (int j = tid; j < nx; j += nt) {
      colx[j] = fmax(fabs(cs * Dx[j] * Dx[j] * (double)q[j]), Ed[j] * Dx[j]);
      rowd[j] = Ed[j] * Dx[j];
    }
    for (int j = tid; j < nu; j += nt) {
      double v = fabs(cs * Du[j] * Du[j] * (double)r[j]);
      v = fmax(v, row_scale(d, j, Du) * Du[j]);  // identity row j
      if (j >= d.n_tau) {
        const int f = (j - d.n_tau) / d.foot_dim, c = (j - d.n_tau) % d.foot_dim;
        const double ef = row_scale(d, d.nu + 4 * f, Du);
        if (c < 2) v = fmax(v, ef * Du[j]);
        if (c == 2) v = fmax(v, ef * mu * Du[j]);
      }
      colu[j] = v;
    }
    __syncthreads();
    // each stage's A_k and B_k go through LDS with coalesced loads; then one
    // thread per A column, per dynamics row and per B column takes the stage's
    // maximum into its own running maximum (no two threads share an accumulator)
    {
      const int role = tid >> 6, idx = tid & 63;
      double acc = 0.0;
      for (int k = 0; k < N; ++k) {
        const T* Ak = in.A + d.oA + (int64_t)k * nx * nx;
        const T* Bk = in.B + d.oB + (int64_t)k * nx * nu;
        for (int e = tid; e < nx * nx; e += nt) sA[e] = Ak[e];
        for (int e = tid; e < nx * nu; e += nt) sB[e] = Bk[e];
        __syncthreads();
        if (role == 0 && idx < nx && k >= 1) {  // column idx of A_k (x_k, k >= 1)
          for (int i = 0; i < nx; ++i) acc = fmax(acc, fabs((double)sA[i * nx + idx]) * Ed[i]);
        } else if (role == 1 && idx < nx) {     // dynamics row idx of stage k
          const double e = Ed[idx];
          if (k >= 1)
            for (int j = 0; j < nx; ++j) acc = fmax(acc, fabs((double)sA[idx * nx + j]) * e * Dx[j]);
          for (int j = 0; j < nu; ++j) acc = fmax(acc, fabs((double)sB[idx * nu + j]) * e * Du[j]);
        } else if (role == 2 && idx < nu) {     // column idx of B_k
          for (int i = 0; i < nx; ++i) acc = fmax(acc, fabs((double)sB[i * nu + idx]) * Ed[i]);
        }
        __syncthreads();
      }
      if (role == 0 && idx < nx) colx[idx] = fmax(colx[idx], acc * Dx[idx]);
      if (role == 1 && idx < nx) rowd[idx] = fmax(rowd[idx], acc);
      if (role == 2 && idx < nu) colu[idx] = fmax(colu[idx], acc * Du[idx]);
    }
    __syncthreads();
    // tied input groups take their largest norm; then divide by the square roots
    double nux = 0.0;
    if (tid < nu) {
      const int g = tie_of(d, tid);
      nux = colu[tid];
      for (int j = 0; j < nu; ++j)
        if (tie_of(d, j) == g) nux = fmax(nux, colu[j]);
    }
    __syncthreads();
    if (tid < nx) {
      Dx[tid] /= sqrt(clamp_norm(colx[tid]));
      Ed[tid] /= sqrt(clamp_norm(rowd[tid]));
    }
    if (tid < nu) Du[tid] /= sqrt(clamp_norm(nux));
    __syncthreads();
    // cost normalisation: mean scaled cost weight over all N (nx + nu) primal
    // columns, and the largest scaled linear cost term
    double part = 0.0, qmax = 0.0;
    for (int j = tid; j < nx; j += nt) {
      part += fabs(cs * Dx[j] * Dx[j] * (double)q[j]) * N;
      for (int k = 1; k <= N; ++k)
        qmax = fmax(qmax, fabs(cs * Dx[j] * ((double)q[j] * (double)xr[k * nx + j])));
    }
    for (int j = tid; j < nu; j += nt) part += fabs(cs * Du[j] * Du[j] * (double)r[j]) * N;
    for (int o = 32; o > 0; o >>= 1) {
      part += __shfl_down(part, o);
      qmax = fmax(qmax, __shfl_down(qmax, o));
    }
    if ((tid & 63) == 0) {
      cpart[tid >> 6] = part;
      cmax[tid >> 6] = qmax;
    }
    __syncthreads();
    if (tid == 0) {  // fixed order: the sum does not depend on timing
      double sum = 0.0, mx = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) {
        sum += cpart[w];
        mx = fmax(mx, cmax[w]);
      }
      const double pn = sum / ((double)N * (nx + nu));
      const double qn = clamp_norm(mx);
      cs = cs / clamp_norm(fmax(pn, qn));
    }
    __syncthreads();
  }
  double* sg = scale + (int64_t)agent * kScaleStride;
  for (int j = tid; j < nx; j += nt) sg[j] = Dx[j];
  for (int j = tid; j < nu; j += nt) sg[kScaleDu + j] = Du[j];
  if (tid == 0) sg[kScaleC] = cs;
  // the scaled problem
  for (int64_t e = tid; e < (int64_t)N * nx * nx; e += nt) {
    const int i = (int)((e / nx) % nx), j = (int)(e % nx);
    out.A[d.oA + e] = (T)((double)in.A[d.oA + e] * Dx[j] / Dx[i]);
  }
  for (int64_t e = tid; e < (int64_t)N * nx * nu; e += nt) {
    const int i = (int)((e / nu) % nx), j = (int)(e % nu);
    out.B[d.oB + e] = (T)((double)in.B[d.oB + e] * Du[j] / Dx[i]);
  }
  for (int e = tid; e < N * nx; e += nt) out.c[d.oc + e] = (T)((double)in.c[d.oc + e] / Dx[e % nx]);
  for (int e = tid; e < (N + 1) * nx; e += nt) out.xr[d.oxr + e] = (T)((double)xr[e] / Dx[e % nx]);
  for (int j = tid; j < nx; j += nt) {
    out.q[d.oq + j] = (T)(cs * Dx[j] * Dx[j] * (double)q[j]);
    out.x0[d.ox0 + j] = (T)((double)in.x0[d.ox0 + j] / Dx[j]);
  }
  for (int j = tid; j < nu; j += nt) out.r[d.orr + j] = (T)(cs * Du[j] * Du[j] * (double)r[j]);
  for (int j = tid; j < d.n_tau; j += nt) out.tau[d.otau + j] = (T)((double)in.tau[d.otau + j] / Du[j]);
  if (tid == 0)
    out.mu[d.omu] = d.n_feet > 0 ? (T)(mu * Du[d.n_tau + 2] / Du[d.n_tau]) : (T)mu;
  // a warm start moves into the scaled variables
  if (agent_warm(warm, d)) {
    for (int e = tid; e < N * nu; e += nt) st.u[d.ou + e] = (T)((double)st.u[d.ou + e] / Du[e % nu]);
    for (int e = tid; e < N * m; e += nt) {
      const double er = row_scale(d, e % m, Du);
      st.z[d.oz + e] = (T)((double)st.z[d.oz + e] * er);
      st.y[d.oy + e] = (T)(cs * (double)st.y[d.oy + e] / er);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_unscale(const AgentDesc* __restrict__ desc, int n, const double* __restrict__ scale, State<T> st) {
  const int agent = blockIdx.x;
  if (agent >= n) return;
  const AgentDesc d = desc[agent];
  const double* sg = scale + (int64_t)agent * kScaleStride;
  const double* Dx = sg;
  const double* Du = sg + kScaleDu;
  const double cs = sg[kScaleC];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < (d.N + 1) * d.nx; e += nt) st.x[d.ox + e] = (T)((double)st.x[d.ox + e] * Dx[e % d.nx]);
  for (int e = tid; e < d.N * d.nu; e += nt) st.u[d.ou + e] = (T)((double)st.u[d.ou + e] * Du[e % d.nu]);
  for (int e = tid; e < d.N * d.m; e += nt) {
    const double er = row_scale(d, e % d.m, Du);
    st.z[d.oz + e] = (T)((double)st.z[d.oz + e] / er);
    st.y[d.oy + e] = (T)((double)st.y[d.oy + e] * er / cs);
  }
}

template <typename T>
__global__ void __launch_bounds__(64)
k_rho_update(const AgentDesc* __restrict__ desc, int n, Inputs<T> in, State<T> st,
             const double* __restrict__ res, double* __restrict__ rho, double tol,
             double* __restrict__ hist, int n_seg, int seg) {
  const int agent = blockIdx.x;
  if (agent >= n) return;
  const AgentDesc d = desc[agent];
  if (st.status[agent] != AGENT_OK) {
    if (threadIdx.x == 0) hist[(int64_t)agent * n_seg + seg] = rho[agent];
    return;
  }
  const int lane = threadIdx.x, N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  const T* q = in.q + d.oq;
  const T* r = in.r + d.orr;
  const double mu = (double)in.mu[d.omu];
  __shared__ double ud[kMaxNu], yd[kMaxNu + 32];
  double cu = 0, zn = 0, px = 0, cty = 0, qn = 0;
  for (int k = 0; k < N; ++k) {
    const T* uk = st.u + d.ou + (int64_t)k * nu;
    const T* zk = st.z + d.oz + (int64_t)k * m;
    const T* yk = st.y + d.oy + (int64_t)k * m;
    __syncthreads();
    for (int j = lane; j < nu; j += 64) ud[j] = (double)uk[j];
    for (int i = lane; i < m; i += 64) yd[i] = (double)yk[i];
    __syncthreads();
    for (int i = lane; i < m; i += 64) {
      cu = fmax(cu, fabs(c_row<double>(d, i, mu, ud)));
      zn = fmax(zn, fabs((double)zk[i]));
    }
    for (int j = lane; j < nu; j += 64) {
      cty = fmax(cty, fabs(ct_row<double>(d, j, mu, yd)));
      px = fmax(px, fabs((double)r[j] * ud[j]));
    }
  }
  for (int e = lane; e < N * nx; e += 64) {
    const int j = e % nx;
    px = fmax(px, fabs((double)q[j] * (double)st.x[d.ox + nx + e]));
    qn = fmax(qn, fabs((double)q[j] * (double)in.xr[d.oxr + nx + e]));
  }
  for (int o = 32; o > 0; o >>= 1) {
    cu = fmax(cu, __shfl_down(cu, o));
    zn = fmax(zn, __shfl_down(zn, o));
    px = fmax(px, __shfl_down(px, o));
    cty = fmax(cty, __shfl_down(cty, o));
    qn = fmax(qn, __shfl_down(qn, o));
  }
  if (lane != 0) return;
  const double tiny = 1e-30;
  const double prim = res[4 * (int64_t)agent] / fmax(fmax(cu, zn), tiny);
  const double dual = res[4 * (int64_t)agent + 1] / fmax(fmax(fmax(px, cty), qn), tiny);
  const double cur = rho[agent];
  double est = cur * sqrt(prim / fmax(dual, tiny));
  est = fmin(fmax(est, kRhoLo), kRhoHi);
  est = exp2(rint(4.0 * log2(est)) / 4.0);
  const double next = (est > tol * cur || est < cur / tol) ? est : cur;
  rho[agent] = next;
  hist[(int64_t)agent * n_seg + seg] = next;
}

__global__ void k_rho_init(double* __restrict__ rho, double* __restrict__ hist, int n, int n_seg,
                           double x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rho[i] = x;
  hist[(int64_t)i * n_seg] = x;
}

}  // namespace

template <typename T>
hipError_t launch_ruiz(const AgentDesc* d_desc, int n, Inputs<T> in, int rounds, ScaledInputs<T> out,
                       double* scale, int warm, State<T> st, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ruiz<T>, dim3(n), dim3(kThreads), 0, stream, d_desc, nullptr, n, in, rounds,
                     out, scale, warm, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unscale(const AgentDesc* d_desc, int n, const double* scale, State<T> st,
                          hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unscale<T>, dim3(n), dim3(kThreads), 0, stream, d_desc, n, scale, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rho_update(const AgentDesc* d_desc, int n, Inputs<T> in, State<T> st,
                             const double* res, double* rho, double tol, double* hist, int n_seg,
                             int seg, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_update<T>, dim3(n), dim3(64), 0, stream, d_desc, n, in, st, res, rho, tol,
                     hist, n_seg, seg);
  return hipGetLastError();
}

hipError_t launch_rho_init(double* rho, double* hist, int n, int n_seg, double x, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_init, dim3((n + 255) / 256), dim3(256), 0, stream, rho, hist, n, n_seg, x);
  return hipGetLastError();
}

#define MPC_SCALING_INSTANTIATE(T)                                                              \
  template hipError_t launch_ruiz<T>(const AgentDesc*, int, Inputs<T>, int, ScaledInputs<T>,     \
                                     double*, int, State<T>, hipStream_t);                       \
  template hipError_t launch_unscale<T>(const AgentDesc*, int, const double*, State<T>,          \
                                        hipStream_t);                                            \
  template hipError_t launch_rho_update<T>(const AgentDesc*, int, Inputs<T>, State<T>,           \
                                           const double*, double*, double, double*, int, int,    \
                                           hipStream_t);
MPC_SCALING_INSTANTIATE(float)
MPC_SCALING_INSTANTIATE(double)

}  // namespace mpc
