// The Riccati factor of the generic path as a parallel-in-time scan over the
// stages (the role of Eq. (ldl) for long horizons served with few agents).
//
// The backward recursion P_k = Qt_k + A_k' P_{k+1} (I + C_k P_{k+1})^{-1} A_k,
// C_k = B_k Rt_k^{-1} B_k' (Rt_k diagonal), P_N = Qt_N, is the composition
// P_k = f_k(f_{k+1}(... f_{N-1}(Qt_N))) of maps f(P) = J + A' P (I + C P)^{-1} A.
// Maps of this form compose within the family: with M = I + C_i J_j,
//   (A, C, J)_i o (A, C, J)_j = (A_j M^{-1} A_i,
//                                A_j M^{-1} C_i A_j' + C_j,
//                                A_i' M^{-T} J_j A_i + J_i),
// an associative product, so every suffix product e_k o ... o e_N (whose J is
// P_k) comes out of ceil(log2(N + 1)) rounds of a doubling scan: in round r
// element k takes e_k o e_{k + 2^r} (if that exists), one workgroup per
// element, every agent and stage of a round in one launch.  The terminal
// element is (0, 0, Qt_N).  Then each stage's operators K_k, A_cl,k, H_k^{-1}
// and s_k follow from P_{k+1} independently (factor_stage, one workgroup per
// stage).  FP64 throughout; the block products of a combine run on the FP64
// matrix cores, the inverse of M by Gauss-Jordan with partial pivoting (M is
// not symmetric; its eigenvalues are those of I + C^{1/2} J C^{1/2}, >= 1).
//
//   k_scan_init    : the stage's row bounds and its element (A_k, C_k, Qt_k);
//                    the stage-0 workgroup checks the agent's inputs and sets
//                    its status;
//   k_scan_combine : one round of the scan (ping-pong buffers);
//   k_scan_ops     : the stage's operators from P_{k+1}.
#include <hip/hip_runtime.h>
#include <math.h>

#include "factor_stage.h"
#include "mpc_internal.h"
#include "stage_rows.h"

namespace mpc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// One 16x16 tile of C = op(A) op(B) (inner dimension K, zero-padded) on the
// FP64 matrix cores; a(i, k), b(k, j) read LDS or global operands.  Element v
// of this lane is C[ti*16 + lane/16 + 4v][tj*16 + lane%16].
template <class FA, class FB>
__device__ inline d4 tile_f64(int ti, int tj, int K, int lane, FA a, FB b) {
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int r = lane & 15, kk = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double av = a(ti * 16 + r, k0 + kk);
    const double bv = b(k0 + kk, tj * 16 + r);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// out(i, j) = sum_t a(i, t) b(t, j) for i, j < n, the tiles spread over the
// workgroup's wavefronts; store(i, j, v) writes one result.
template <class FA, class FB, class FS>
__device__ inline void product(int n, int tid, int nt, FA a, FB b, FS store) {
  const int tiles = (n + 15) / 16, wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
  for (int t = wave; t < tiles * tiles; t += nw) {
    const int ti = t / tiles, tj = t % tiles;
    const d4 acc = tile_f64(ti, tj, n, lane, a, b);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + (lane >> 4) + 4 * v, j = tj * 16 + (lane & 15);
      if (i < n && j < n) store(i, j, acc[v]);
    }
  }
}

__device__ inline int64_t elem_off(int slot, int Nmax, int k, int nx) {
  return ((int64_t)slot * (Nmax + 1) + k) * 3 * nx * nx;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_scan_init(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int Nmax,
            Inputs<T> in, SolverConsts sc_all, T* __restrict__ ws, double* __restrict__ E,
            int32_t* __restrict__ status) {
  const int slot = blockIdx.x / (Nmax + 1), k = blockIdx.x % (Nmax + 1);
  const int a = list[slot];
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, nu = d.nu, m = d.m;
  if (k > N) return;
  const SolverConsts sc = agent_consts(sc_all, a);
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Bk = reinterpret_cast<double*>(smem_raw);  // nx*nu
  double* rhok = Bk + nx * nu;                          // m
  double* irdg = rhok + m;                              // 1 / diag Rt_k, nu
  __shared__ int s_flag;
  if (k == 0) {
    if (tid == 0) s_flag = 0;
    __syncthreads();
    if (!agent_inputs_ok(in, d, tid, nt)) atomicOr(&s_flag, 1);
    __syncthreads();
    if (tid == 0) status[a] = s_flag ? AGENT_NONFINITE : AGENT_OK;
  }
  const T* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  double* Ae = E + elem_off(slot, Nmax, k, nx);
  double* Ce = Ae + nx * nx;
  double* Je = Ce + nx * nx;
  // Qt_k: the state weight with its penalties (and the no-slip rows' weight)
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    Je[idx] = ((i == j) ? (double)in.q[d.oq + i] + sc.sigma + state_rho<double>(in, d, i, sc) : 0.0) +
              contact_weight<double>(in, d, k, i, j, sc);
  }
  if (k == N) {
    for (int idx = tid; idx < nx * nx; idx += nt) {
      Ae[idx] = 0.0;
      Ce[idx] = 0.0;
    }
    return;
  }
  // the stage's row bounds (as the serial factor writes them)
  T* wl = ws + d.ows + (int64_t)N * (nu * nx + nx * nx + nu * nu + nx);
  T* wh = wl + (int64_t)N * m;
  T* wrho = wh + (int64_t)N * m;
  for (int i = tid; i < m; i += nt) {
    T lo, hi, rr;
    row_bounds<T, T>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rr);
    wl[(int64_t)k * m + i] = lo;
    wh[(int64_t)k * m + i] = hi;
    wrho[(int64_t)k * m + i] = rr;
    double dl, dh;
    row_bounds<double, T>(d, i, stance + k * d.n_feet, tau, sc, dl, dh, rhok[i]);
  }
  const T* Bg = in.B + d.oB + (int64_t)k * nx * nu;
  for (int idx = tid; idx < nx * nu; idx += nt) Bk[idx] = (double)Bg[idx];
  __syncthreads();
  for (int j = tid; j < nu; j += nt)
    irdg[j] = 1.0 / rtilde_diag<double, double>(d, j, (double)in.r[d.orr + j], (double)in.mu[d.omu], rhok, sc);
  __syncthreads();
  const T* Ag = in.A + d.oA + (int64_t)k * nx * nx;
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    Ae[idx] = (double)Ag[idx];
    double acc = 0.0;
    for (int t = 0; t < nu; ++t) acc += Bk[i * nu + t] * irdg[t] * Bk[j * nu + t];
    Ce[idx] = acc;
  }
}

// LDS of a combine: A_i, C_i, A_j, J_j, the augmented [M | I] (nx x 2nx) and
// one more nx x nx buffer, plus the pivot bookkeeping.
__host__ __device__ inline size_t combine_lds_bytes(int nx) {
  return (size_t)8 * (4 * nx * nx + 2 * nx * nx + nx * nx + nx);
}

__global__ void __launch_bounds__(256)
k_scan_combine(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int Nmax, int dist,
               const double* __restrict__ Ein, double* __restrict__ Eout,
               const int32_t* __restrict__ status) {
  const int slot = blockIdx.x / (Nmax + 1), k = blockIdx.x % (Nmax + 1);
  const int a = list[slot];
  const AgentDesc d = desc[a];
  const int N = d.N, nx = d.nx, n2 = nx * nx;
  if (k > N || status[a] != AGENT_OK) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* ei = Ein + elem_off(slot, Nmax, k, nx);
  double* eo = Eout + elem_off(slot, Nmax, k, nx);
  if (k + dist > N) {  // nothing to compose with this round
    for (int idx = tid; idx < 3 * n2; idx += nt) eo[idx] = ei[idx];
    return;
  }
  const double* ej = Ein + elem_off(slot, Nmax, k + dist, nx);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Ai = reinterpret_cast<double*>(smem_raw);
  double* Ci = Ai + n2;
  double* Aj = Ci + n2;
  double* Jj = Aj + n2;
  double* aug = Jj + n2;    // nx x 2nx: [M | I] -> [I | M^-1]
  double* Tb = aug + 2 * n2;
  double* fcol = Tb + n2;   // column factors of a Gauss-Jordan step
  __shared__ int s_piv;
  __shared__ double s_pv;
  const int la = 2 * nx;
  for (int idx = tid; idx < n2; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    Ai[idx] = ei[idx];
    Ci[idx] = 0.5 * (ei[n2 + idx] + ei[n2 + j * nx + i]);
    Aj[idx] = ej[idx];
    Jj[idx] = 0.5 * (ej[2 * n2 + idx] + ej[2 * n2 + j * nx + i]);
  }
  __syncthreads();
  // [I + C_i J_j | I]
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Ci[i * nx + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Jj[t * nx + j] : 0.0; },
          [&](int i, int j, double v) { aug[i * la + j] = v + (i == j ? 1.0 : 0.0); });
  for (int idx = tid; idx < n2; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    aug[i * la + nx + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // Gauss-Jordan with partial pivoting
  for (int p = 0; p < nx; ++p) {
    if (tid < 64) {
      double best = -1.0;
      int bi = p;
      for (int r = p + tid; r < nx; r += 64) {
        const double v = fabs(aug[r * la + p]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) s_piv = bi;
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != p)
      for (int j = tid; j < la; j += nt) {
        const double t = aug[p * la + j];
        aug[p * la + j] = aug[pr * la + j];
        aug[pr * la + j] = t;
      }
    __syncthreads();
    if (tid == 0) s_pv = 1.0 / aug[p * la + p];
    for (int r = tid; r < nx; r += nt) fcol[r] = aug[r * la + p];
    __syncthreads();
    const double ip = s_pv;
    for (int j = tid; j < la; j += nt) aug[p * la + j] *= ip;
    __syncthreads();
    for (int idx = tid; idx < nx * la; idx += nt) {
      const int r = idx / la, j = idx % la;
      if (r != p) aug[idx] -= fcol[r] * aug[p * la + j];
    }
    __syncthreads();
  }
  const double* Mi = aug + nx;  // M^-1, row stride la
  double* T1 = aug;              // the left half is free now
  // T1 = A_j M^-1
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Aj[i * nx + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Mi[t * la + j] : 0.0; },
          [&](int i, int j, double v) { Tb[i * nx + j] = v; });
  __syncthreads();
  // A_out = T1 A_i ; Tb -> T1 (left half of aug) first so that Tb is free
  for (int idx = tid; idx < n2; idx += nt) T1[(idx / nx) * la + idx % nx] = Tb[idx];
  __syncthreads();
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? T1[i * la + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Ai[t * nx + j] : 0.0; },
          [&](int i, int j, double v) { eo[i * nx + j] = v; });
  // X = T1 C_i
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? T1[i * la + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Ci[t * nx + j] : 0.0; },
          [&](int i, int j, double v) { Tb[i * nx + j] = v; });
  __syncthreads();
  // C_out = X A_j' + C_j
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Tb[i * nx + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Aj[j * nx + t] : 0.0; },
          [&](int i, int j, double v) { eo[n2 + i * nx + j] = v + ej[n2 + i * nx + j]; });
  __syncthreads();
  // W = M^-T J_j (into Tb), then Y = W A_i (into T1), J_out = A_i' Y + J_i
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Mi[t * la + i] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Jj[t * nx + j] : 0.0; },
          [&](int i, int j, double v) { Tb[i * nx + j] = v; });
  __syncthreads();
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Tb[i * nx + t] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? Ai[t * nx + j] : 0.0; },
          [&](int i, int j, double v) { T1[i * la + j] = v; });
  __syncthreads();
  product(nx, tid, nt, [&](int i, int t) { return i < nx && t < nx ? Ai[t * nx + i] : 0.0; },
          [&](int t, int j) { return t < nx && j < nx ? T1[t * la + j] : 0.0; },
          [&](int i, int j, double v) { eo[2 * n2 + i * nx + j] = v + ei[2 * n2 + i * nx + j]; });
}

template <typename T>
__global__ void __launch_bounds__(256)
k_scan_ops(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int Nmax, Inputs<T> in,
           SolverConsts sc_all, T* __restrict__ ws, const double* __restrict__ E,
           int32_t* __restrict__ status) {
  const int slot = blockIdx.x / Nmax, k = blockIdx.x % Nmax;
  const int a = list[slot];
  const AgentDesc d = desc[a];
  const int nx = d.nx, nu = d.nu;
  if (k >= d.N || status[a] != AGENT_OK) return;
  const SolverConsts sc = agent_consts(sc_all, a);
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the serial factor's LDS layout
  double* H = reinterpret_cast<double*>(smem_raw);
  double* P = H + nu * nu;
  double* Ak = P + nx * nx;
  double* PA = Ak + nx * nx;
  double* Bk = PA + nx * nx;
  double* PB = Bk + nx * nu;
  double* G = PB + nx * nu;
  double* rdg = G + nu * nx;
  double* rhok = rdg + nu;
  __shared__ int s_flag;
  if (tid == 0) s_flag = 0;
  // P_{k+1}: the J of the suffix product from stage k + 1, symmetrised
  const double* J = E + elem_off(slot, Nmax, k + 1, nx) + 2 * nx * nx;
  for (int idx = tid; idx < nx * nx; idx += nt) {
    const int i = idx / nx, j = idx % nx;
    P[idx] = 0.5 * (J[idx] + J[j * nx + i]);
  }
  __syncthreads();
  const FactorLds<double> F{H, P, Ak, PA, Bk, PB, G, rdg, rhok};
  if (!factor_stage<T>(in, sc, d, k, F, ws, &s_flag, false, tid, nt) && tid == 0)
    atomicMax(status + a, (int32_t)AGENT_NOT_PD);
}

}  // namespace

size_t scan_elements_bytes(int n_agents, int Nmax, int nx) {
  return (size_t)n_agents * (Nmax + 1) * 3 * nx * nx * sizeof(double);
}

template <typename T>
hipError_t launch_scan_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, int Nmax, int nx,
                              int nu, int m, Inputs<T> in, SolverConsts sc, T* ws, double* E0, double* E1,
                              int32_t* status, size_t lds_ops, hipStream_t s) {
  if (n_launch <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)n_launch * (Nmax + 1);
  hipLaunchKernelGGL(k_scan_init<T>, dim3(blocks), dim3(256), (size_t)8 * (nx * nu + m + nu), s, d_desc,
                     list, Nmax, in, sc, ws, E0, status);
  hipError_t e = hipGetLastError();
  double* src = E0;
  double* dst = E1;
  for (int dist = 1; e == hipSuccess && dist < Nmax + 1; dist *= 2) {
    hipLaunchKernelGGL(k_scan_combine, dim3(blocks), dim3(256), combine_lds_bytes(nx), s, d_desc, list, Nmax,
                       dist, src, dst, status);
    e = hipGetLastError();
    double* t = src;
    src = dst;
    dst = t;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_ops<T>, dim3((unsigned)n_launch * Nmax), dim3(256), lds_ops, s, d_desc, list,
                     Nmax, in, sc, ws, src, status);
  return hipGetLastError();
}

hipError_t scan_set_limits() {
  // nx <= 48 (the planner rejects larger states for this factor)
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_scan_combine),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)combine_lds_bytes(48));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_scan_ops<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_scan_ops<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64);
  return e;
}

template hipError_t launch_scan_factor<float>(const AgentDesc*, const int32_t*, int, int, int, int, int,
                                              Inputs<float>, SolverConsts, float*, double*, double*,
                                              int32_t*, size_t, hipStream_t);
template hipError_t launch_scan_factor<double>(const AgentDesc*, const int32_t*, int, int, int, int, int,
                                               Inputs<double>, SolverConsts, double*, double*, double*,
                                               int32_t*, size_t, hipStream_t);

}  // namespace mpc
