// Register-resident FP32 solve: two kernels, one workgroup per agent.
//
// k_riccati (once per solve) -- the Riccati factor that plays the role of
// Eq. (ldl): stage by stage, k = N-1 .. 0, in FP64 in LDS.  The dense block
// products (P B, P A, B'PB, B'PA, H^{-1} G, A'PA + G'K, A + B K) run on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64, 16x16 tiles spread over the
// workgroup's wavefronts); the stage Hessian is inverted in FP64 by one
// wavefront.  Stage k's operators A_cl,k, K_k, B_k, H_k^{-1} are rounded to
// float once and written to HBM already in the per-lane order of the
// register layout below, so the iteration kernel loads them with coalesced
// loads: opws[agent][stage][slot][lane], SLOTS floats per lane.
//
// k_admm_resident -- the QP iterations of Alg. 1 (the role of
// Eqs. (backsolve_1)-(backsolve_2), then projection and dual update) with
// every operator on chip: one stage wavefront per stage keeps K_k, B_k and
// H_k^{-1} in registers and runs the work that is independent across stages
// (linear terms, input step, relaxation / projection / dual update); one
// chain wavefront runs both serial chains alone (p_k = g_k + A_cl,k' p'_k
// backwards, x_{k+1} = A_cl,k x_k + e_k forwards), reading A_cl,k from LDS,
// with no workgroup barrier between hops.  The two kinds of wavefront hand
// over through per-stage progress flags in LDS (value = iteration number):
// a stage wavefront starts its input step as soon as p'_k is flagged and its
// state update as soon as x_k is.  The chain wavefront turns p'_0 into x_1
// itself, x_1 = A_cl,0 x_0 + g'_0 + S_0 p'_0 with S_0 = -B_0 H_0^{-1} B_0'
// from the factor (per agent, after the stage slots and s_k) and
// g'_0 = c_0 - B_0 H_0^{-1} rt_0 from stage 0's wavefront, formed before p'_0.
// Every product (chain hops and stage-parallel products) sums its per-lane
// block and its cross-lane butterfly in FP32; the ADMM state (x, u, z, y),
// the offsets added to the sums and the relaxation / projection / dual update
// are FP64.
//
// k_admm_stream -- the same iterations for horizons 12 to 20: one stage
// wavefront per two stages, the chain wavefront, and a loader wavefront that
// streams A_cl,k from HBM through a ring of LDS slots in the order the chain
// consumes them.
//
// Register layout of a stage's operators (lane = 8a + b, a, b in 0..7):
//   Acl[i][j] = A_cl[a*RB + i][b*RB + j]      RB = ceil(nx/8)
//   Km[i][j]  = K[b*CB + i][a*RB + j]         CB = ceil(nu/8)
//   Bm[i][j]  = B[a*RB + i][b*CB + j]
//   Hm[i][j]  = H^{-1}[a*CB + i][b*CB + j]
// so every product is a small per-lane block followed by a butterfly over
// either the b index (lanes xor 1, 2, 4) or the a index (lanes xor 8, 16, 32).
#include <math.h>

#include <type_traits>

#include "fused.h"
#include "stage_rows.h"
#include "xlane.h"

namespace mpc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxStages = 12;   // wavefronts per iteration workgroup (stages + chain)
constexpr int kFactorWaves = 8;  // wavefronts per factor workgroup

template <int NX, int NU>
struct FS {
  static constexpr int RB = (NX + 7) / 8, CB = (NU + 7) / 8;
  static constexpr int NXP = 8 * RB, NUP = 8 * CB;  // padded vector lengths
  static constexpr int NXT = (NX + 15) / 16 * 16;   // MFMA-padded sizes
  static constexpr int NUT = (NU + 15) / 16 * 16;
  static constexpr int LX = NXT + 1, LU = NUT + 1;  // odd strides: no bank conflicts
  static constexpr int AQ = (RB * RB + 3) / 4;  // float4 quads of the chain operator
  static constexpr int SLOTS = 4 * AQ + CB * RB + RB * CB + CB * CB;
  static constexpr int MMAX = 64;
};


// Hides a uniform integer's value from the optimiser, so addresses built on it
// are formed once instead of folded into others with negative offsets.
__device__ inline void opaque_s(int& v) { asm volatile("" : "+s"(v)); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// v + (the same register of the lane 16 or 32 lanes away): permlane swaps hand
// each lane its partner's value; both lanes of a pair add in the same order.
__device__ inline float swap_sum16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap_sum32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double join(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double swap_sum16(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  return join(l[0], h[0]) + join(l[1], h[1]);
}
__device__ inline double swap_sum32(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  return join(l[0], h[0]) + join(l[1], h[1]);
}

// All-reduce over the 8 lanes 8a .. 8a+7 (the b index): quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror.  Every lane ends with the same sum.
template <typename T>
__device__ inline T red_b(T v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  return v;
}
// All-reduce over the 8 lanes b, b+8, .., b+56 (the a index): row_ror 8, then
// the 16- and 32-lane swaps.
template <typename T>
__device__ inline T red_a(T v) {
  v += dpp<0x128>(v);
  v = swap_sum16(v);
  v = swap_sum32(v);
  return v;
}

// One 16x16 output tile of C = op(A) op(B) on the FP64 matrix cores.
// a(i, k) and b(k, j) read the (padded, zero-filled) operands from LDS.
// Output element v of this lane is C[ti*16 + lane/16 + 4*v][tj*16 + lane%16].
template <class FA, class FB>
__device__ inline d4 mfma_tile(int ti, int tj, int K, int lane, FA a, FB b) {
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int r = lane & 15, kk = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double av = a(ti * 16 + r, k0 + kk);
    const double bv = b(k0 + kk, tj * 16 + r);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Product precision of the factor's block products: FP64 (v_mfma_f64_16x16x4f64),
// BF16 / FP16 operands with FP32 accumulation (v_mfma_f32_16x16x32_{bf16,f16}),
// or FP32 operands (v_mfma_f32_16x16x4f32).
enum { kProdF64 = 0, kProdBF16 = 1, kProdF16 = 2, kProdF32 = 3 };

// Output row of element v of this lane in a 16x16 tile (column is lane % 16).
template <int PREC>
__device__ inline int orow(int lane, int v) {
  return PREC == kProdF64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

// One 16x16 tile of C = op(A) op(B) over K (zero beyond K) in precision PREC.
// Low precision: lane l feeds A[row l%16][k0 + 8(l/16) ..+7] and
// B[k0 + 8(l/16) ..+7][col l%16]; operands are rounded to nearest from the
// LDS doubles, products are exact and accumulate in FP32.
template <int PREC, class FA, class FB>
__device__ inline d4 prod_tile(int ti, int tj, int K, int lane, FA a, FB b) {
  if constexpr (PREC == kProdF64) {
    return mfma_tile(ti, tj, K, lane, a, b);
  } else if constexpr (PREC == kProdF32) {
    // lane l feeds A[row l%16][k0 + l/16] and B[k0 + l/16][col l%16]
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, kk = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 4) {
      const float av = (float)(k0 + kk < K ? a(ti * 16 + r, k0 + kk) : 0.0);
      const float bv = (float)(k0 + kk < K ? b(k0 + kk, tj * 16 + r) : 0.0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    return d4{(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]};
  } else {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 32) {
      if constexpr (PREC == kProdBF16) {
        bf16x8 av, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int kk = k0 + 8 * g + i;
          av[i] = (__bf16)(float)(kk < K ? a(ti * 16 + r, kk) : 0.0);
          bv[i] = (__bf16)(float)(kk < K ? b(kk, tj * 16 + r) : 0.0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      } else {
        f16x8 av, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int kk = k0 + 8 * g + i;
          av[i] = (_Float16)(float)(kk < K ? a(ti * 16 + r, kk) : 0.0);
          bv[i] = (_Float16)(float)(kk < K ? b(kk, tj * 16 + r) : 0.0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
      }
    }
    return d4{(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]};
  }
}

// ------------------------------------------------------------------------------------
// Riccati factor (FP64, MFMA)
// ------------------------------------------------------------------------------------

// The t-th tile on or above the diagonal of a TT x TT grid of tiles, row by row
// (t < TT (TT + 1) / 2).
__device__ inline void upper_tile(int t, int TT, int& ti, int& tj) {
  ti = 0;
  while (ti < TT - 1 && t >= TT - ti) {
    t -= TT - ti;
    ++ti;
  }
  tj = ti + t;
}

// LDS of the factor kernel (doubles unless noted): three NXT x LX buffers
// (P_{k+1} -> G -> K -> P_k; A_k -> A_cl,k; P A_k), one NXT x LU buffer
// (P B_k -> H_k -> H_k^{-1}), B_k as float, and small vectors.  Under 80 KB for
// the shapes built here, so two workgroups share a compute unit.
template <int NX, int NU>
constexpr int riccati_lds_bytes() {
  using S = FS<NX, NU>;
  return 8 * (3 * S::NXT * S::LX + S::NXT * S::LU + S::NUT + S::MMAX + S::NXT + 8 * S::NUT) +
         4 * S::NXT * S::LU + 16;
}

// P += Jc' diag(rho_c,k) Jc, the no-slip rows' term of stage k's state weight
// (P: NX x NX at row stride LX): the rows' penalties first into rc (LDS, nc
// doubles), then each entry's nc-term sum with a block of Jc's loads in flight
// (indices past nc clamped, terms added in increasing row order).  Ends with a
// workgroup barrier.
template <int NX>
__device__ inline void add_contact_weight(double* P, int LX, const Inputs<float>& in, const AgentDesc& d,
                                          int k, const SolverConsts& sc, double* rc, int tid, int nt) {
  const int nc = d.n_feet * d.foot_dim;
  const float* Jc = in.J + d.oJ;
  const uint8_t* stance = in.st + d.ost;
  for (int r = tid; r < nc; r += nt) {
    double rr;
    contact_row(d, stance, k, r, sc, rr);
    rc[r] = rr;
  }
  __syncthreads();
  for (int e = tid; e < NX * NX; e += nt) {
    const int i = e / NX, j = e % NX;
    double acc = 0.0;
    for (int r0 = 0; r0 < nc; r0 += 8) {
      float ji[8], jj[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int r = min(r0 + t, nc - 1);
        ji[t] = Jc[r * NX + i];
        jj[t] = Jc[r * NX + j];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (r0 + t < nc) acc += (double)ji[t] * rc[r0 + t] * (double)jj[t];
    }
    P[i * LX + j] += acc;
  }
  __syncthreads();
}

// RES: operators go to the register-resident layout at fws + ofw (FP64
// products, or FP32 products for MPC_FP32_MFMA).
// Otherwise (mixed precision, or FP64 products for the generic iteration
// kernel at any horizon) they go to the generic per-agent layout at fws + ows:
// K [N][nu][nx], A_cl [N][nx][nx], H^{-1} [N][nu][nu], s [N][nx], then l, h,
// rho [N][m].
//
// Stage k: PB = P B_k, PA = P A_k, s_k = P c_k; H_k = Rt_k + B_k' PB and
// G = B_k' PA; H_k^{-1}; K_k = -H_k^{-1} G; A_cl,k = A_k + B_k K_k; operators
// out; then P_k = Q + sigma I + PA' A_cl,k (= Q + A'PA + G'K, as P is
// symmetric), formed on and above the diagonal and mirrored.
template <int NX, int NU, int PREC, bool RES>
__global__ void __launch_bounds__(64 * kFactorWaves, PREC == kProdF64 || (PREC == kProdF32 && (RES || NX == 48)) ? 4 : 2)
k_riccati(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
          Inputs<float> in, SolverConsts sc_all, float* __restrict__ fws, int32_t* __restrict__ status) {
  using S = FS<NX, NU>;
  constexpr int RB = S::RB, CB = S::CB, NXP = S::NXP, NXT = S::NXT, NUT = S::NUT;
  constexpr int LX = S::LX, LU = S::LU, SLOTS = S::SLOTS;
  static_assert(riccati_lds_bytes<NX, NU>() <= 80 * 1024, "two workgroups per compute unit");
  if ((int)blockIdx.x >= n_launch) return;
  const int agent = list ? list[blockIdx.x] : (int)blockIdx.x;
  const SolverConsts sc = agent_consts(sc_all, agent);
  const AgentDesc d = desc[agent];
  const int N = d.N, M = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = tid >> 6, lane = tid & 63;
  const int nw = nt >> 6;
  extern __shared__ __align__(16) unsigned char sm[];
  double* P = reinterpret_cast<double*>(sm);  // P_{k+1} | G_k | K_k | P_k   NXT x LX
  double* G = P;
  double* Kd = P;
  double* Ak = P + NXT * LX;                  // A_k, then A_cl,k           NXT x LX
  double* PA = Ak + NXT * LX;                 // P A_k                      NXT x LX
  double* PB = PA + NXT * LX;                 // P B_k, then H_k, H_k^{-1}  NXT x LU
  double* H = PB;
  double* rdg = PB + NXT * LU;                // diag Rt_k                  NUT
  double* rhok = rdg + NUT;                   // row penalties              MMAX
  double* ck = rhok + S::MMAX;                // c_k                        NXT
  double* xcol = ck + NXT;                    // Gauss-Jordan pivot column / row exchange
  double* xrow = xcol + 4 * NUT;              //   (two buffers of 2 NUT each)
  float* Bk = reinterpret_cast<float*>(xrow + 4 * NUT);  // B_k (float, exact)  NXT x LU
  int* flag = reinterpret_cast<int*>(Bk + NXT * LU);

  const float* A = in.A + d.oA;
  const float* B = in.B + d.oB;
  const float* c = in.c + d.oc;
  const float* q = in.q + d.oq;
  const float* r = in.r + d.orr;
  const float* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const float muf = in.mu[d.omu];
  const double mu = (double)muf;
  constexpr bool kResident = RES;
  static_assert(!RES || PREC == kProdF64 || PREC == kProdF32,
                "the register-resident path takes FP64 or FP32 products");
  float* ops = fws + (kResident ? d.ofw : d.ows);
  float* sk_out = kResident ? ops + (int64_t)N * SLOTS * 64  // [stage][NXP]
                            : ops + (int64_t)N * (NU * NX + NX * NX + NU * NU);
  float* gK = ops;
  float* gAcl = gK + (int64_t)N * NU * NX;
  float* gHi = gAcl + (int64_t)N * NX * NX;
  float* gl = sk_out + (int64_t)N * NX;
  float* gh = gl + (int64_t)N * M;
  float* grho = gh + (int64_t)N * M;

  for (int i = tid; i < riccati_lds_bytes<NX, NU>() / 4; i += nt) reinterpret_cast<int*>(sm)[i] = 0;
  __syncthreads();
  // non-finite inputs mark the agent and stop it (A_k and B_k are checked as
  // each stage's prefetch lands, below)
  bool ok = isfinite(muf);
  for (int i = tid; i < N * NX; i += nt) ok &= (bool)isfinite(c[i]);
  for (int i = tid; i < (N + 1) * NX; i += nt) ok &= (bool)isfinite(in.xr[d.oxr + i]);
  for (int i = tid; i < NX; i += nt) ok &= (bool)isfinite(q[i]) && (bool)isfinite(in.x0[d.ox0 + i]);
  for (int i = tid; i < NU; i += nt) ok &= (bool)isfinite(r[i]);
  for (int i = tid; i < d.n_tau; i += nt) ok &= (bool)isfinite(tau[i]);
  if (in.uref)
    for (int i = tid; i < N * NU; i += nt) ok &= (bool)isfinite(in.uref[d.our + i]);
  if (in.xlo)  // joint limits: no NaN bound, and an interval that is not empty
    for (int i = tid; i < NX; i += nt) {
      const float lo = in.xlo[d.oq + i], hi = in.xhi[d.oq + i];
      ok &= !isnan(lo) && !isnan(hi) && lo <= hi;
    }
  if (in.J)  // no-slip rows: a finite foot Jacobian
    for (int i = tid; i < d.n_feet * d.foot_dim * NX; i += nt) ok &= (bool)isfinite(in.J[d.oJ + i]);
  if (!ok) atomicOr(flag, 1);
  // state weight Q + sigma I (+ the joint-limit rows' penalties, + the no-slip
  // rows' dense Jc' diag(rho_c,N) Jc)
  for (int i = tid; i < NX; i += nt) P[i * LX + i] = (double)q[i] + sc.sigma + state_rho<double>(in, d, i, sc);
  if (in.J) {
    __syncthreads();
    add_contact_weight<NX>(P, LX, in, d, N, sc, xcol, tid, nt);
  }
  __syncthreads();
  if (flag[0]) {
    if (tid == 0) status[agent] = AGENT_NONFINITE;
    return;
  }

  // A_k and B_k of the next stage are fetched into registers one stage ahead,
  // so their global-load latency hides behind the current stage.
  constexpr int kT = 64 * kFactorWaves;
  constexpr int PFA = (NX * NX + kT - 1) / kT, PFB = (NX * NU + kT - 1) / kT;
  float pfa[PFA], pfb[PFB];
  auto prefetch = [&](int kk) {
    const float* Ag = A + (int64_t)kk * NX * NX;
    const float* Bg = B + (int64_t)kk * NX * NU;
#pragma unroll
    for (int t = 0; t < PFA; ++t) pfa[t] = tid + t * kT < NX * NX ? Ag[tid + t * kT] : 0.f;
#pragma unroll
    for (int t = 0; t < PFB; ++t) pfb[t] = tid + t * kT < NX * NU ? Bg[tid + t * kT] : 0.f;
  };
  prefetch(N - 1);
  for (int k = N - 1; k >= 0; --k) {
    bool fin = true;
#pragma unroll
    for (int t = 0; t < PFA; ++t) {
      const int i = tid + t * kT;
      if (i < NX * NX) {
        Ak[(i / NX) * LX + i % NX] = (double)pfa[t];
        fin &= (bool)isfinite(pfa[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < PFB; ++t) {
      const int i = tid + t * kT;
      if (i < NX * NU) {
        Bk[(i / NU) * LU + i % NU] = pfb[t];
        fin &= (bool)isfinite(pfb[t]);
      }
    }
    if (!fin) atomicOr(flag, 1);
    if (k > 0) prefetch(k - 1);
    for (int i = tid; i < M; i += nt) {
      double lo, hi;
      row_bounds<double, float>(d, i, stance + k * d.n_feet, tau, sc, lo, hi, rhok[i]);
      if (!kResident) {
        gl[k * M + i] = (float)lo;
        gh[k * M + i] = (float)hi;
        grho[k * M + i] = (float)rhok[i];
      }
    }
    for (int i = tid; i < NX; i += nt) ck[i] = (double)c[(int64_t)k * NX + i];
    __syncthreads();
    if (flag[0]) {  // a non-finite A_k or B_k (every thread reads the same flag)
      if (tid == 0) status[agent] = AGENT_NONFINITE;
      return;
    }
    for (int j = tid; j < NUT; j += nt)
      rdg[j] = j < NU ? rtilde_diag<double, double>(d, j, (double)r[j], mu, rhok, sc) : 1.0;
    // PB = P B_k (NXT x NUT) and PA = P A_k (NXT x NXT); s_k = P c_k
    {
      constexpr int TB = (NXT / 16) * (NUT / 16), TA = (NXT / 16) * (NXT / 16);
      for (int t = w; t < TB + TA; t += nw) {
        if (t < TB) {
          const int ti = t / (NUT / 16), tj = t % (NUT / 16);
          d4 acc = prod_tile<PREC>(ti, tj, NXT, lane, [&](int i, int kk) { return P[i * LX + kk]; },
                                   [&](int kk, int j) { return (double)Bk[kk * LU + j]; });
#pragma unroll
          for (int v = 0; v < 4; ++v)
            PB[(ti * 16 + orow<PREC>(lane, v)) * LU + tj * 16 + (lane & 15)] = acc[v];
        } else {
          const int tt = t - TB, ti = tt / (NXT / 16), tj = tt % (NXT / 16);
          d4 acc = prod_tile<PREC>(ti, tj, NXT, lane, [&](int i, int kk) { return P[i * LX + kk]; },
                                   [&](int kk, int j) { return Ak[kk * LX + j]; });
#pragma unroll
          for (int v = 0; v < 4; ++v)
            PA[(ti * 16 + orow<PREC>(lane, v)) * LX + tj * 16 + (lane & 15)] = acc[v];
        }
      }
      const int sstride = kResident ? NXP : NX;
      for (int i = tid; i < sstride; i += nt) {
        double acc = 0.0;
        if (i < NX)
          for (int t = 0; t < NX; ++t) acc += P[i * LX + t] * ck[t];
        sk_out[k * sstride + i] = (float)acc;
      }
    }
    __syncthreads();
    // H = diag(Rt_k) + B_k' PB (NUT x NUT), held in registers until PB is
    // dead; G = B_k' PA (NUT x NXT) over the dead P_{k+1}
    {
      constexpr int TH = (NUT / 16) * (NUT / 16), TG = (NUT / 16) * (NXT / 16);
      static_assert(TH <= kFactorWaves, "one H tile per wavefront at most");
      d4 hacc = {0.0, 0.0, 0.0, 0.0};
      // H tiles on the wavefronts past the G tiles (wrapping), so the two
      // products spread over all wavefronts
      const int hw = (w - TG + 2 * nw) % nw;
      const int hti = hw / (NUT / 16), htj = hw % (NUT / 16);
      if (hw < TH)
        hacc = prod_tile<PREC>(hti, htj, NXT, lane, [&](int i, int kk) { return (double)Bk[kk * LU + i]; },
                               [&](int kk, int j) { return PB[kk * LU + j]; });
      for (int t = w; t < TG; t += nw) {
        const int ti = t / (NXT / 16), tj = t % (NXT / 16);
        d4 acc = prod_tile<PREC>(ti, tj, NXT, lane, [&](int i, int kk) { return (double)Bk[kk * LU + i]; },
                                 [&](int kk, int j) { return PA[kk * LX + j]; });
#pragma unroll
        for (int v = 0; v < 4; ++v)
          G[(ti * 16 + orow<PREC>(lane, v)) * LX + tj * 16 + (lane & 15)] = acc[v];
      }
      __syncthreads();
      if (hw < TH)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = hti * 16 + orow<PREC>(lane, v), j = htj * 16 + (lane & 15);
          H[i * LU + j] = hacc[v] + (i == j ? rdg[i] : 0.0);
        }
    }
    __syncthreads();
    // H_k^{-1} in place by block Gauss-Jordan sweeps without pivoting over the
    // padded NUT x NUT matrix, eliminating the 2x2 pivot block
    // P = H[j..j+1][j..j+1] per sweep for j < NU (the padding is an identity
    // block with zero coupling: no sweep changes it, and it is its own inverse):
    //   P <- P^{-1},  H[p][o] <- P^{-1} H[p][o],  H[o][p] <- -H[o][p] P^{-1},
    //   H[o][o] <- H[o][o] - H[o][p] P^{-1} H[p][o].
    // H_k is SPD, so every pivot block is SPD (a Schur complement); a pivot
    // block that is not (P00 <= 0 or det P <= 0) means H_k is not positive
    // definite.  Every thread keeps two entries of one row (an even column
    // pair, so both lie inside or both outside a pivot block) in registers;
    // each sweep publishes the pivot rows and columns through a
    // double-buffered LDS exchange, so one barrier per sweep orders a
    // buffer's writes after its previous readers.
    {
      static_assert(NUT * NUT == 2 * 64 * kFactorWaves, "two entries per thread");
      constexpr int TPR = NUT / 2;  // threads per row
      const int row = tid / TPR, c0 = (tid % TPR) * 2;
      double h0 = H[row * LU + c0], h1 = H[row * LU + c0 + 1];
      bool bad = false;
      static_assert(NU % 2 == 0, "2x2 pivot blocks");
      for (int j = 0; j < NU; j += 2) {
        double* xc = xcol + ((j >> 1) & 1) * 2 * NUT;  // [row][2]: columns j, j+1
        double* xr = xrow + ((j >> 1) & 1) * 2 * NUT;  // [2][col]: rows j, j+1
        if (c0 == j) {
          xc[2 * row] = h0;
          xc[2 * row + 1] = h1;
        }
        if ((row >> 1) == (j >> 1)) {
          xr[(row - j) * NUT + c0] = h0;
          xr[(row - j) * NUT + c0 + 1] = h1;
        }
        __syncthreads();
        const double a = xr[j], b = xr[j + 1], dd = xr[NUT + j + 1];
        const double det = a * dd - b * b;
        if (!(a > 0.0) || !(det > 0.0)) {  // the same values in every thread: a uniform exit
          bad = true;
          break;
        }
        const double id = 1.0 / det;
        const double i00 = dd * id, i01 = -b * id, i11 = a * id;  // P^{-1} (symmetric)
        const bool rp = (row >> 1) == (j >> 1), cp = c0 == j;
        if (rp && cp) {
          const int t = row - j;
          h0 = t == 0 ? i00 : i01;
          h1 = t == 0 ? i01 : i11;
        } else if (rp) {
          const int t = row - j;
          const double w0 = t == 0 ? i00 : i01, w1 = t == 0 ? i01 : i11;
          h0 = w0 * xr[c0] + w1 * xr[NUT + c0];
          h1 = w0 * xr[c0 + 1] + w1 * xr[NUT + c0 + 1];
        } else {
          const double q0 = xc[2 * row], q1 = xc[2 * row + 1];
          const double v0 = q0 * i00 + q1 * i01, v1 = q0 * i01 + q1 * i11;  // H[o][p] P^{-1}
          if (cp) {
            h0 = -v0;
            h1 = -v1;
          } else {
            h0 -= v0 * xr[c0] + v1 * xr[NUT + c0];
            h1 -= v0 * xr[c0 + 1] + v1 * xr[NUT + c0 + 1];
          }
        }
      }
      if (bad) {
        if (tid == 0) flag[1] = 1;
      } else {
        H[row * LU + c0] = h0;
        H[row * LU + c0 + 1] = h1;
      }
    }
    __syncthreads();
    if (flag[1]) {
      if (tid == 0) status[agent] = AGENT_NOT_PD;
      return;
    }
    // K_k = -H_k^{-1} G (NUT x NXT, FP64) in place of G: every tile is held in
    // registers until all of G has been read
    {
      constexpr int TK = (NUT / 16) * (NXT / 16);
      static_assert(TK <= kFactorWaves, "one K tile per wavefront");
      const int ti = w / (NXT / 16), tj = w % (NXT / 16);
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      if (w < TK)
        acc = mfma_tile(ti, tj, NUT, lane,
                        [&](int i, int kk) { return (i < NU && kk < NU) ? H[i * LU + kk] : 0.0; },
                        [&](int kk, int j) { return G[kk * LX + j]; });
      __syncthreads();
      if (w < TK)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Kd[(ti * 16 + (lane >> 4) + 4 * v) * LX + tj * 16 + (lane & 15)] = -acc[v];
    }
    __syncthreads();
    // A_cl,k = A_k + B_k K_k in place of A_k (each entry read and written by one lane)
    {
      constexpr int TA = (NXT / 16) * (NXT / 16);
      for (int t = w; t < TA; t += nw) {
        const int ti = t / (NXT / 16), tj = t % (NXT / 16);
        d4 acc = prod_tile<PREC>(ti, tj, NUT, lane, [&](int i, int kk) { return (double)Bk[i * LU + kk]; },
                                 [&](int kk, int j) { return Kd[kk * LX + j]; });
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = ti * 16 + orow<PREC>(lane, v), j = tj * 16 + (lane & 15);
          Ak[i * LX + j] += acc[v];
        }
      }
    }
    __syncthreads();
    // P_k = Q + sigma I + PA' A_cl,k (= Q + sigma I + A'PA - G'H^{-1}G, symmetric):
    // the tiles on and above the diagonal only, into registers here and into
    // the P buffer (over the dead K_k) once the operators below are written;
    // each value goes to both of its mirror positions
    constexpr int TT = NXT / 16, TU = TT * (TT + 1) / 2;
    constexpr int PR = (TU + kFactorWaves - 1) / kFactorWaves;
    d4 pacc[PR];
#pragma unroll
    for (int rr = 0; rr < PR; ++rr) {
      const int t = w + rr * kFactorWaves;
      pacc[rr] = d4{0.0, 0.0, 0.0, 0.0};
      if (t >= TU) continue;
      int ti, tj;
      upper_tile(t, TT, ti, tj);
      pacc[rr] = prod_tile<PREC>(ti, tj, NXT, lane, [&](int i, int kk) { return PA[kk * LX + i]; },
                                   [&](int kk, int j) { return Ak[kk * LX + j]; });
    }
    // stage k's operators, rounded to float, in register-layout order (or in
    // the generic row-major layout for the mixed-precision iterations)
    if (!kResident) {
      for (int e = tid; e < NU * NX; e += nt) gK[(int64_t)k * NU * NX + e] = (float)Kd[(e / NX) * LX + e % NX];
      for (int e = tid; e < NX * NX; e += nt) gAcl[(int64_t)k * NX * NX + e] = (float)Ak[(e / NX) * LX + e % NX];
      for (int e = tid; e < NU * NU; e += nt) gHi[(int64_t)k * NU * NU + e] = (float)H[(e / NU) * LU + e % NU];
    }
    float* dst = ops + (int64_t)k * SLOTS * 64;
    constexpr int AQ = S::AQ;
    for (int e = tid; kResident && e < SLOTS * 64; e += nt) {
      double v = 0.0;
      if (e < AQ * 256) {
        // A_cl,k as [quad][lane][4], slot i*RB + j; the lane roles of a and b
        // swap on odd stages
        const int slot = 4 * (e >> 8) + (e & 3), ln = (e >> 2) & 63;
        const int a = (k & 1) ? ln & 7 : ln >> 3, b = (k & 1) ? ln >> 3 : ln & 7;
        const int ri = a * RB + slot / RB, cj = b * RB + slot % RB;
        if (slot < RB * RB && ri < NX && cj < NX) v = Ak[ri * LX + cj];
        dst[e] = (float)v;
        continue;
      }
      const int slot = (e >> 6) - 4 * AQ, ln = e & 63, a = ln >> 3, b = ln & 7;
      if (slot < CB * RB) {
        const int ri = b * CB + slot / RB, cj = a * RB + slot % RB;
        if (ri < NU && cj < NX) v = Kd[ri * LX + cj];
      } else if (slot < 2 * CB * RB) {
        const int sl = slot - CB * RB, ri = a * RB + sl / CB, cj = b * CB + sl % CB;
        if (ri < NX && cj < NU) v = (double)Bk[ri * LU + cj];
      } else {
        const int sl = slot - 2 * CB * RB, ri = a * CB + sl / CB, cj = b * CB + sl % CB;
        if (ri < NU && cj < NU) v = H[ri * LU + cj];
      }
      dst[e] = (float)v;
    }
    __syncthreads();  // the last reads of K_k are done
#pragma unroll
    for (int rr = 0; rr < PR; ++rr) {
      const int t = w + rr * kFactorWaves;
      if (t >= TU) continue;
      int ti, tj;
      upper_tile(t, TT, ti, tj);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + orow<PREC>(lane, v), j = tj * 16 + (lane & 15);
        if (ti == tj && i > j) continue;
        const double pv =
            pacc[rr][v] + ((i == j && i < NX) ? (double)q[i] + sc.sigma + state_rho<double>(in, d, i, sc) : 0.0);
        P[i * LX + j] = pv;
        P[j * LX + i] = pv;
      }
    }
    __syncthreads();
    // the no-slip rows' dense Jc' diag(rho_c,k) Jc
    if (in.J && k > 0) add_contact_weight<NX>(P, LX, in, d, k, sc, xcol, tid, nt);
  }
  if (kResident) {
    // S_0 = -B_0 H_0^{-1} B_0' (FP64 matrix-core tiles, once per agent), written in
    // the chain operator order of an even stage: x~_1 = A_cl,0 x~_0 + c_0
    // - B_0 H_0^{-1} rt_0 + S_0 p'_0, so the iterations' chain wavefront forms
    // x~_1 from p'_0 in one product.  W = B_0 H_0^{-1} over P A_k and S_0 over P,
    // neither of which stage 0 needs any more.
    double* W = PA;
    double* S0 = P;
    constexpr int TW = (NXT / 16) * (NUT / 16), TS = (NXT / 16) * (NXT / 16);
    for (int t = w; t < TW; t += nw) {
      const int ti = t / (NUT / 16), tj = t % (NUT / 16);
      const d4 acc = mfma_tile(ti, tj, NUT, lane,
                               [&](int i, int kk) { return kk < NU ? (double)Bk[i * LU + kk] : 0.0; },
                               [&](int kk, int j) { return (kk < NU && j < NU) ? H[kk * LU + j] : 0.0; });
#pragma unroll
      for (int v = 0; v < 4; ++v) W[(ti * 16 + (lane >> 4) + 4 * v) * LU + tj * 16 + (lane & 15)] = acc[v];
    }
    __syncthreads();
    for (int t = w; t < TS; t += nw) {
      const int ti = t / (NXT / 16), tj = t % (NXT / 16);
      const d4 acc = mfma_tile(ti, tj, NUT, lane, [&](int i, int kk) { return W[i * LU + kk]; },
                               [&](int kk, int j) { return kk < NU ? (double)Bk[j * LU + kk] : 0.0; });
#pragma unroll
      for (int v = 0; v < 4; ++v) S0[(ti * 16 + (lane >> 4) + 4 * v) * LX + tj * 16 + (lane & 15)] = -acc[v];
    }
    __syncthreads();
    float* s0 = ops + (int64_t)N * (SLOTS * 64 + S::NXP);
    for (int e = tid; e < S::AQ * 256; e += nt) {
      const int slot = 4 * (e >> 8) + (e & 3), ln = (e >> 2) & 63;
      const int ri = (ln >> 3) * RB + slot / RB, cj = (ln & 7) * RB + slot % RB;
      s0[e] = (slot < RB * RB && ri < NX && cj < NX) ? (float)S0[ri * LX + cj] : 0.f;
    }
  }
  if (tid == 0) status[agent] = AGENT_OK;
}

// ------------------------------------------------------------------------------------
// ADMM iterations: N stage wavefronts with register-resident operators and one
// chain wavefront
// ------------------------------------------------------------------------------------

// Progress flags between the chain wavefront and the stage wavefronts, in
// LDS: each holds the number of the last iteration (from 1) whose data it
// covers, is set after that data is stored (and after the setter's last read
// of data it hands back), and is polled with acquire order before the data is
// read.  Layout: g_k ready (A), p'_k ready
// (backward chain), e_k ready (C), xt_k ready (forward chain), abort.
constexpr int kSyncG = 0, kSyncP = kMaxStages, kSyncE = 2 * kMaxStages, kSyncX = 3 * kMaxStages;

// Role of hardware wavefront hw of a register-resident iteration workgroup
// (stage roles 0 .. chain-1, the chain wavefront `chain`, idle roles past
// it).  A CU places a workgroup's wavefronts on its four SIMDs in turn
// (wavefronts 3, 7, 11 share one), so the chain goes to wavefront 3, which
// then shares its SIMD with fewer stage wavefronts than the last wavefront
// would for N = 6, 8, 9, 10; the stage roles keep their order on the others.
// (Measured: 5.17 -> 5.09 ms per launch at N = 10.  The streaming kernel keeps
// its order: there the same move made every horizon slower.)
__device__ inline int wave_role(int hw, int chain) {
  if (chain < 3) return hw;
  if (hw == 3) return chain;
  const int r = hw < 3 ? hw : hw - 1;
  return r >= chain ? r + 1 : r;
}
constexpr int kSyncAbort = 4 * kMaxStages + 1, kSyncInts = 4 * kMaxStages + 2;
constexpr int kSpinLimit = 1 << 21;  // polls of one wait (about 0.1 s)

// Setting a flag does not wait for the wavefront's earlier LDS stores to
// complete.  This rests on the CDNA memory model for LDS: the LDS unit
// executes the DS instructions of one wavefront in the order they were issued
// (which is also why LGKM_CNT counts LDS-only traffic down in order), so the
// data stores are performed before the flag store, and a reader that sees the
// flag and then loads sees the data.  The compiler-level barrier keeps the
// stores before the flag in issue order.  A release store would add an
// s_waitcnt lgkmcnt(0) before every flag on the critical path.
__device__ inline void flag_set(int* f, int v) {
  asm volatile("" ::: "memory");
  __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Waits until every one of f[0 .. n) (n <= 64, one lane each) is >= v.  The
// first polls spin (the handovers on the critical path are short); later ones
// sleep between polls.  The wait is bounded: past kSpinLimit polls it raises
// the abort flag, and every wait returns at once while that flag is up (it is
// read every 64 polls), so the workgroup always drains (the agent then reports
// non-finite).
__device__ inline void flag_wait(int* f, int n, int v, int* abort, int lane) {
  for (int t = 0; t < kSpinLimit; ++t) {
    const int x = lane < n ? __hip_atomic_load(f + lane, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) : v;
    if (__all(x >= v)) return;
    if ((t & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    if (t >= 32) __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct IterLds {
  int acl, xtf, ppf, gf, ef, sf, cf;                               // float
  int xd, ud, zd, yd, lod, hid, rhod, irhod, wvd, rtd, dd, utd, qd, xrd, qtd, bvd;  // double
  int jc, jac, dnf;                                                // float, no-slip rows
  int zcd, ycd, wcd, rcd, ircd;                                    // double, no-slip rows
  int flag, sync, total;
};

// nc: no-slip rows per state (0 without them)
template <int NX, int NU>
__host__ __device__ inline IterLds iter_lds_layout(int N, int M, int nc = 0) {
  using S = FS<NX, NU>;
  IterLds L{};
  int o = 0;
  auto take = [&](int bytes) {
    const int r = o;
    o += (bytes + 15) & ~15;
    return r;
  };
  L.acl = take(4 * N * S::AQ * 256);
  L.xtf = take(4 * (N + 1) * S::NXP);
  L.ppf = take(4 * N * S::NXP);
  L.gf = take(4 * N * S::NXP);
  L.ef = take(4 * N * S::NXP);
  L.sf = take(4 * N * S::NXP);
  L.cf = take(4 * N * S::NXP);
  L.xd = take(8 * (N + 1) * S::NXP);
  L.ud = take(8 * N * S::NUP);
  L.zd = take(8 * N * M);
  L.yd = take(8 * N * M);
  L.lod = take(8 * N * M);
  L.hid = take(8 * N * M);
  L.rhod = take(8 * N * M);
  L.irhod = take(8 * N * M);
  L.wvd = take(8 * N * M);
  L.rtd = take(8 * N * S::NUP);
  L.dd = take(8 * N * S::NUP);
  L.utd = take(8 * N * S::NUP);
  L.qd = take(8 * S::NXP);
  L.xrd = take(8 * (N + 1) * S::NXP);
  L.qtd = take(8 * N * S::NXP);
  L.bvd = take(8 * S::NXP);
  L.jc = take(4 * nc * S::NXP);
  L.jac = take(4 * nc * S::NXP);
  L.dnf = take(nc ? 4 * S::NXP : 0);
  L.zcd = take(8 * N * nc);
  L.ycd = take(8 * N * nc);
  L.wcd = take(8 * N * nc);
  L.rcd = take(8 * N * nc);
  L.ircd = take(8 * N * nc);
  L.flag = take(16);
  L.sync = take(4 * kSyncInts);
  L.total = o;
  return L;
}

// red_a of every element of v[0..n): pairs share their 16- and 32-lane swaps
// (a reduce-scatter of the pair, then a gather back), 3.5 swaps and adds per
// value instead of 6.
template <int n>
__device__ inline void red_a_all(float (&v)[n]) {
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] += dpp<0x128>(v[i]);
#pragma unroll
  for (int i = 0; i + 1 < n; i += 2) {
    // rows (16 lanes) of v[i] = X0..X3, of v[i+1] = Y0..Y3
    const auto r1 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 1]), false, false);
    const float s = __uint_as_float(r1[0]) + __uint_as_float(r1[1]);  // X0+X1, Y0+Y1, X2+X3, Y2+Y3
    const auto r2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    const float t = __uint_as_float(r2[0]) + __uint_as_float(r2[1]);  // X, Y, X, Y
    const auto r3 = __builtin_amdgcn_permlane16_swap(__float_as_uint(t), __float_as_uint(t), false, false);
    v[i] = __uint_as_float(r3[0]);      // X in every row
    v[i + 1] = __uint_as_float(r3[1]);  // Y in every row
  }
  if (n & 1) v[n - 1] = swap_sum32(swap_sum16(v[n - 1]));
}

// R consecutive floats from / to LDS, in float2 pieces when R is even (the
// callers' offsets are then even)
template <int R>
__device__ inline void lds_load(float (&v)[R], const float* p) {
  if constexpr (R % 2 == 0) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const float2 t = reinterpret_cast<const float2*>(p)[i];
      v[2 * i] = t.x;
      v[2 * i + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = p[i];
  }
}
template <int R>
__device__ inline void lds_store(float* p, const float (&v)[R]) {
  if constexpr (R % 2 == 0) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) reinterpret_cast<float2*>(p)[i] = make_float2(v[2 * i], v[2 * i + 1]);
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) p[i] = v[i];
  }
}

// A_cl,k of the chain wavefront, one float4 quad at a time from LDS
// ([stage][quad][lane][4]); slot i*RB + j of the lane's RB x RB block.
template <int AQ>
__device__ inline void load_chain_op(float (&M)[4 * AQ], const float4* acl4, int kk, int lane) {
  int off = kk * AQ * 64;  // opaque: one base, then immediate offsets
  asm volatile("" : "+s"(off));
  const float4* src = acl4 + off + lane;
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const float4 v = src[q * 64];
    M[4 * q] = v.x;
    M[4 * q + 1] = v.y;
    M[4 * q + 2] = v.z;
    M[4 * q + 3] = v.w;
  }
}

// x^0 = rollout of the exact dynamics x_{k+1} = A_k x_k + B_k u_k + c_k from x_0
// under u^0, by the whole workgroup: quad qq owns state row qq (its lanes every
// fourth column), the rows of stages k+1..k+3 are in flight while stage k is
// summed.  xd [N+1][NXP] (x_0 set) and ud [N][NUP] in LDS; one barrier per stage.
// For the streaming kernel, whose LDS holds a few stages' operators at a time
// (the register-resident kernel rolls out through A_cl in LDS and the stage
// wavefronts' B_k, K_k instead, reading no A_k or B_k).
template <int NX, int NU>
__device__ inline void rollout_exact(const float* __restrict__ A, const float* __restrict__ B,
                                     const float* __restrict__ c, double* xd, const double* ud, int N,
                                     int tid, int nt) {
  using S = FS<NX, NU>;
  constexpr int NXP = S::NXP, NUP = S::NUP;
  constexpr int TA = (NX + 3) / 4, TB = (NU + 3) / 4;
  const int qq = tid >> 2, sub = tid & 3;
  if ((nt >> 2) < NX) {
    // a workgroup with fewer quads than state rows (the shortest horizons):
    // rows in turn, nothing prefetched
    for (int kk = 0; kk < N; ++kk) {
      for (int r = qq; r < NX; r += nt >> 2) {
        const float* Ar = A + ((int64_t)kk * NX + r) * NX;
        const float* Br = B + ((int64_t)kk * NX + r) * NU;
        double acc = 0.0;
        for (int t = sub; t < NX; t += 4) acc += (double)Ar[t] * xd[kk * NXP + t];
        for (int t = sub; t < NU; t += 4) acc += (double)Br[t] * ud[kk * NUP + t];
        acc = quad_sum(acc);
        if (sub == 0) xd[(kk + 1) * NXP + r] = (double)c[(int64_t)kk * NX + r] + acc;
      }
      __syncthreads();
    }
    return;
  }
  const bool row = qq < NX;
  auto load = [&](float (&a)[TA], float (&b)[TB], float& cv, int kk) __attribute__((always_inline)) {
    const float* Ar = A + ((int64_t)kk * NX + (row ? qq : 0)) * NX;
    const float* Br = B + ((int64_t)kk * NX + (row ? qq : 0)) * NU;
#pragma unroll
    for (int t = 0; t < TA; ++t) a[t] = (row && sub + 4 * t < NX) ? Ar[sub + 4 * t] : 0.f;
#pragma unroll
    for (int t = 0; t < TB; ++t) b[t] = (row && sub + 4 * t < NU) ? Br[sub + 4 * t] : 0.f;
    cv = row ? c[(int64_t)kk * NX + qq] : 0.f;
  };
  auto step = [&](const float (&a)[TA], const float (&b)[TB], float cv, int kk) __attribute__((always_inline)) {
    if (row) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < TA; ++t)
        if (sub + 4 * t < NX) acc += (double)a[t] * xd[kk * NXP + sub + 4 * t];
#pragma unroll
      for (int t = 0; t < TB; ++t)
        if (sub + 4 * t < NU) acc += (double)b[t] * ud[kk * NUP + sub + 4 * t];
      acc = quad_sum(acc);
      if (sub == 0) xd[(kk + 1) * NXP + qq] = (double)cv + acc;
    }
    __syncthreads();
  };
  float a0[TA], b0[TB], a1[TA], b1[TB], a2[TA], b2[TB], c0 = 0.f, c1 = 0.f, c2 = 0.f;
  load(a0, b0, c0, 0);
  if (N > 1) load(a1, b1, c1, 1);
  if (N > 2) load(a2, b2, c2, 2);
  for (int kk = 0; kk < N; kk += 3) {
    step(a0, b0, c0, kk);
    if (kk + 3 < N) load(a0, b0, c0, kk + 3);
    if (kk + 1 < N) {
      step(a1, b1, c1, kk + 1);
      if (kk + 4 < N) load(a1, b1, c1, kk + 4);
    }
    if (kk + 2 < N) {
      step(a2, b2, c2, kk + 2);
      if (kk + 5 < N) load(a2, b2, c2, kk + 5);
    }
  }
}

// Stage wavefront k (k < N) keeps K_k, B_k and H_k^{-1} in registers and runs
// everything that is independent across stages; the chain wavefront (the
// last one) runs both serial chains alone, streaming A_cl,k from LDS one stage
// ahead, with no barrier between hops.  Its operators alternate lane roles
// with the stage's parity (even k: rows a*RB + i, columns b*RB + j; odd k:
// rows b*RB + i, columns a*RB + j), so the butterfly of one hop leaves its
// output vector spread over the lanes exactly as the next hop reads it.  Inside
// the iteration loop the two kinds of wavefront meet only through the
// progress flags; workgroup barriers separate the set-up, the iterations and
// the write-out.  ROWS: the instantiation that takes the no-slip rows (the
// other one carries none of their code).
template <int NX, int NU, bool ROWS = false>
__device__ __forceinline__ void admm_resident_agent(const AgentDesc* __restrict__ desc, int agent,
                                                    Inputs<float> in, SolverConsts sc_all, int iters,
                                                    int warm, const float* __restrict__ fws,
                                                    State<float> st) {
  using S = FS<NX, NU>;
  constexpr int RB = S::RB, CB = S::CB, NXP = S::NXP, NUP = S::NUP, SLOTS = S::SLOTS, AQ = S::AQ;
  const SolverConsts sc = agent_consts(sc_all, agent);
  const AgentDesc d = desc[agent];
  const int N = d.N, M = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = wave_role(tid >> 6, N), lane = tid & 63, la = lane >> 3, lb = lane & 7;
  float* X = st.x + d.ox;
  float* U = st.u + d.ou;
  float* Z = st.z + d.oz;
  float* Y = st.y + d.oy;
  // no-slip rows J_f v_k = 0 of x_1..x_N (plans with them; N >= 2)
  const int nc = ROWS && in.J ? d.n_feet * d.foot_dim : 0;
  if (st.status[agent] != AGENT_OK) {
    for (int i = tid; i < (N + 1) * d.nx; i += nt) X[i] = NAN;
    for (int i = tid; i < N * d.nu; i += nt) U[i] = NAN;
    for (int i = tid; i < N * M; i += nt) {
      Z[i] = NAN;
      Y[i] = NAN;
    }
    for (int i = tid; i < N * nc; i += nt) {
      st.zc[d.ozc + i] = NAN;
      st.yc[d.ozc + i] = NAN;
    }
    return;
  }
  const IterLds L = iter_lds_layout<NX, NU>(N, M, nc);
  extern __shared__ __align__(16) unsigned char sm[];
  const float4* acl4 = reinterpret_cast<const float4*>(sm + L.acl);
  float* xtf = reinterpret_cast<float*>(sm + L.xtf);
  float* ppf = reinterpret_cast<float*>(sm + L.ppf);
  float* gf = reinterpret_cast<float*>(sm + L.gf);
  float* ef = reinterpret_cast<float*>(sm + L.ef);
  float* sf = reinterpret_cast<float*>(sm + L.sf);
  float* cf = reinterpret_cast<float*>(sm + L.cf);
  double* xd = reinterpret_cast<double*>(sm + L.xd);
  double* ud = reinterpret_cast<double*>(sm + L.ud);
  double* zd = reinterpret_cast<double*>(sm + L.zd);
  double* yd = reinterpret_cast<double*>(sm + L.yd);
  double* lod = reinterpret_cast<double*>(sm + L.lod);
  double* hid = reinterpret_cast<double*>(sm + L.hid);
  double* rhod = reinterpret_cast<double*>(sm + L.rhod);
  double* irhod = reinterpret_cast<double*>(sm + L.irhod);
  double* wvd = reinterpret_cast<double*>(sm + L.wvd);
  double* rtd = reinterpret_cast<double*>(sm + L.rtd);
  double* dd = reinterpret_cast<double*>(sm + L.dd);
  double* utd = reinterpret_cast<double*>(sm + L.utd);
  double* qd = reinterpret_cast<double*>(sm + L.qd);
  double* xrd = reinterpret_cast<double*>(sm + L.xrd);
  double* qtd = reinterpret_cast<double*>(sm + L.qtd);
  double* bvd = reinterpret_cast<double*>(sm + L.bvd);
  // after the x^0 rollout: g'_0 of iterations of odd / even number
  float* g0f = reinterpret_cast<float*>(sm + L.bvd);
  // no-slip rows: Jc [nc][NXP], Jc A_cl,N-1 [nc][NXP], Jc' w_c,N [NXP];
  // z_c, y_c, w_c = y_c - rho_c z_c of x_1..x_N [N][nc]
  float* jc = reinterpret_cast<float*>(sm + L.jc);
  float* jac = reinterpret_cast<float*>(sm + L.jac);
  float* dnf = reinterpret_cast<float*>(sm + L.dnf);
  double* zcd = reinterpret_cast<double*>(sm + L.zcd);
  double* ycd = reinterpret_cast<double*>(sm + L.ycd);
  double* wcd = reinterpret_cast<double*>(sm + L.wcd);
  // the rows' penalties rho_c, negated for the equality (stance) rows
  double* rcd = reinterpret_cast<double*>(sm + L.rcd);
  double* ircd = reinterpret_cast<double*>(sm + L.ircd);  // 1 / rho_c
  int* flag = reinterpret_cast<int*>(sm + L.flag);
  int* sync = reinterpret_cast<int*>(sm + L.sync);

  const float* c = in.c + d.oc;
  const float* q = in.q + d.oq;
  const float* r = in.r + d.orr;
  const float* xr = in.xr + d.oxr;
  const float* x0 = in.x0 + d.ox0;
  const float* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const float* uref = in.uref ? in.uref + d.our : nullptr;
  const double mu = (double)in.mu[d.omu];

  // per-agent vectors into LDS (padding zero), A_cl of every stage into LDS
  // (which it fills whole: the zeroing starts past it), eight float4 loads in
  // flight per thread
  for (int i = L.xtf / 4 + tid; i < L.total / 4; i += nt) reinterpret_cast<int*>(sm)[i] = 0;
  {
    const f4* src = reinterpret_cast<const f4*>(fws + d.ofw);
    f4* dst = reinterpret_cast<f4*>(sm + L.acl);
    const int total = N * AQ * 64;
    constexpr int kBatch = 8;
    for (int i0 = tid; i0 < total; i0 += kBatch * nt) {
      f4 v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int i = i0 + u * nt;
        const int kk = i / (AQ * 64);
        if (i < total) v[u] = src[(int64_t)kk * SLOTS * 16 + (i - kk * AQ * 64)];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int i = i0 + u * nt;
        if (i < total) dst[i] = v[u];
      }
    }
  }
  __syncthreads();
  const float* sk = fws + d.ofw + (int64_t)N * SLOTS * 64;
  for (int i = tid; i < N * NXP; i += nt) sf[i] = sk[i];
  for (int i = tid; i < N * NX; i += nt) cf[(i / NX) * NXP + i % NX] = c[i];
  for (int i = tid; i < NX; i += nt) {
    qd[i] = (double)q[i];
    xd[i] = (double)x0[i];
    xtf[i] = x0[i];
  }
  for (int i = tid; i < (N + 1) * NX; i += nt) xrd[(i / NX) * NXP + i % NX] = (double)xr[i];
  for (int i = tid; i < N * M; i += nt) {
    const int k = i / M, j = i % M;
    double lo, hi, rr;
    row_bounds<double, float>(d, j, stance + k * d.n_feet, tau, sc, lo, hi, rr);
    lod[i] = lo;
    hid[i] = hi;
    rhod[i] = rr;
    irhod[i] = 1.0 / rr;
  }
  const bool wm = agent_warm(warm, d);
  for (int i = tid; i < N * NU; i += nt) ud[(i / NU) * NUP + i % NU] = wm ? (double)U[i] : 0.0;
  for (int i = tid; i < N * M; i += nt) {
    zd[i] = wm ? (double)Z[i] : 0.0;
    yd[i] = wm ? (double)Y[i] : 0.0;
  }
  if (nc) {
    const float* Jc = in.J + d.oJ;
    for (int i = tid; i < nc * NX; i += nt) jc[(i / NX) * NXP + i % NX] = Jc[i];
    for (int i = tid; i < N * nc; i += nt) {
      const double zz = wm ? (double)st.zc[d.ozc + i] : 0.0, yy = wm ? (double)st.yc[d.ozc + i] : 0.0;
      double rr;
      const bool eq = contact_row(d, stance, i / nc + 1, i % nc, sc, rr);
      zcd[i] = zz;
      ycd[i] = yy;
      wcd[i] = yy - rr * zz;
      rcd[i] = eq ? -rr : rr;
      ircd[i] = 1.0 / rr;
    }
  }
  __syncthreads();
  if (nc) {
    // Jc A_cl,N-1: the rows of x_N = A_cl,N-1 x_{N-1} + e_{N-1} as seen from the
    // last stage, so that its wavefront handles them (A_cl,N-1 read from the
    // chain operator layout: slot i*RB + j of lane a*8 + b, or b*8 + a on odd
    // stages, holds row a*RB + i, column b*RB + j)
    const float* aclf = reinterpret_cast<const float*>(sm + L.acl);
    const int kl = N - 1;
    for (int e = tid; e < nc * NX; e += nt) {
      const int rw = e / NX, cj = e % NX, b = cj / RB, j = cj % RB;
      double acc = 0.0;
      for (int ri = 0; ri < NX; ++ri) {
        const int a = ri / RB, slot = (ri % RB) * RB + j, ln = (kl & 1) ? b * 8 + a : a * 8 + b;
        acc += (double)jc[rw * NXP + ri] * (double)aclf[((kl * AQ + (slot >> 2)) * 64 + ln) * 4 + (slot & 3)];
      }
      jac[rw * NXP + cj] = (float)acc;
    }
    __syncthreads();
  }



  const double sigma = sc.sigma, alpha = sc.alpha, oma = 1.0 - sc.alpha;
  const int k = w;  // a stage wavefront's stage

  if (w == N) {
    // ---------------- chain wavefront ----------------
    float M0[4 * AQ], M1[4 * AQ];  // even / odd stage operators
    // x^0 rollout: x_{k+1} = A_cl,k x_k + [B_k (u_k - K_k x_k) + c_k from stage wavefront k]
    for (int kk = 0; kk < N; ++kk) {
      __syncthreads();
      if ((kk & 1) == 0) {
        load_chain_op<AQ>(M0, acl4, kk, lane);
        double sx[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          sx[i] = 0.0;
#pragma unroll
          for (int j = 0; j < RB; ++j) sx[i] += (double)(M0[i * RB + j] * (float)xd[kk * NXP + lb * RB + j]);
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const double v = red_b(sx[i]);
          const int idx = la * RB + i;
          if (lb == 0 && idx < NX) xd[(kk + 1) * NXP + idx] = bvd[idx] + v;
        }
      } else {
        load_chain_op<AQ>(M1, acl4, kk, lane);
        double sx[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          sx[i] = 0.0;
#pragma unroll
          for (int j = 0; j < RB; ++j) sx[i] += (double)(M1[i * RB + j] * (float)xd[kk * NXP + la * RB + j]);
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const double v = red_a(sx[i]);
          const int idx = lb * RB + i;
          if (la == 0 && idx < NX) xd[(kk + 1) * NXP + idx] = bvd[idx] + v;
        }
      }
      __syncthreads();
    }
    __builtin_amdgcn_s_setprio(2);
    // Layout of the backward chain's first input (stage N-1) and of the
    // forward chain's last output: a*RB + i for an even stage, b*RB + i odd.
    const int pidx = ((N - 1) & 1) ? lb * RB : la * RB;
    // p_N = -Q x_ref,N - sigma x_N, from the relaxed x_N (here the rollout's)
    float pN[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
      pN[i] = (float)(-qd[pidx + i] * xrd[N * NXP + pidx + i] - sigma * xd[N * NXP + pidx + i]);
    // A_cl,0 x_0 does not change: the first forward hop only adds e_0
    float ax0[RB];
    {
      load_chain_op<AQ>(M0, acl4, 0, lane);
      float x0v[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) x0v[j] = xtf[lb * RB + j];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        ax0[i] = 0.f;
#pragma unroll
        for (int j = 0; j < RB; ++j) ax0[i] += M0[i * RB + j] * x0v[j];
        ax0[i] = red_b(ax0[i]);
      }
    }
    // A_cl,0 is not read again (x^0 and A_cl,0 x_0 are done): its LDS slot
    // takes S_0, which the backward chain's last hop then prefetches into M0
    {
      const float4* s0 = reinterpret_cast<const float4*>(fws + d.ofw + (int64_t)N * (SLOTS * 64 + NXP));
      float4* acl_w = reinterpret_cast<float4*>(sm + L.acl);
      float4 v[AQ];
#pragma unroll
      for (int q = 0; q < AQ; ++q) v[q] = s0[q * 64 + lane];
#pragma unroll
      for (int q = 0; q < AQ; ++q) acl_w[q * 64 + lane] = v[q];
    }
    float p0[RB];  // p'_0 of the current iteration, on a*RB + i

    for (int it = 0; it < iters; ++it) {
      const int T = it + 1;
      // backward chain, k = N-1 .. 0: p'_k = p_{k+1} + s_k, stored and flagged;
      // p_k = g_k + A_cl,k' p'_k.  p_N is this wavefront's own, so the first hop's
      // product runs before g_{N-1} (the last stage's A) is waited for.  Every
      // hop issues its loads (g_k, s_{k-1}, the next operator) first.
      {
        float pv[RB];  // p'_k of the coming hop, in its input layout
        // Hop kk (first: the first hop of the chain, which waits for the g_k
        // only after its product).  ODD: p'_k on b*RB + i, product summed over
        // b, p_k on a*RB + j; even: the roles of a and b swap.
        auto hop = [&](int kk, bool first, auto odd_c) {
          constexpr bool ODD = decltype(odd_c)::value;
          const int in_idx = ODD ? lb * RB : la * RB, out_idx = ODD ? la * RB : lb * RB;
          // stage offsets kept opaque so each vector is one base plus immediates
          int ok = kk * NXP, om = (kk - 1) * NXP;
          opaque_s(ok);
          opaque_s(om);
          if ((ODD ? la : lb) == 0) lds_store<RB>(ppf + ok + in_idx, pv);
          flag_set(sync + kSyncP + kk, T);  // C_kk may start now
          float gv[RB], sv[RB], qv[RB];
          lds_load<RB>(sv, sf + om + out_idx);
          lds_load<RB>(gv, gf + ok + out_idx);  // (reloaded below on the first hop)
#pragma unroll
          for (int j = 0; j < RB; ++j) qv[j] = 0.f;
          if constexpr (ODD) {
            load_chain_op<AQ>(M0, acl4, kk - 1, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
              for (int j = 0; j < RB; ++j) qv[j] += M1[i * RB + j] * pv[i];
#pragma unroll
            for (int j = 0; j < RB; ++j) qv[j] = red_b(qv[j]);
          } else {
            load_chain_op<AQ>(M1, acl4, kk - 1, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
              for (int j = 0; j < RB; ++j) qv[j] += M0[i * RB + j] * pv[i];
            red_a_all<RB>(qv);
          }
          if (first) {
            flag_wait(sync + kSyncG, N, T, sync + kSyncAbort, lane);
            lds_load<RB>(gv, gf + ok + out_idx);
          }
#pragma unroll
          for (int j = 0; j < RB; ++j) pv[j] = gv[j] + qv[j] + sv[j];
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        int kk = N - 1;
#pragma unroll
        for (int i = 0; i < RB; ++i) pv[i] = pN[i] + sf[kk * NXP + pidx + i];
        bool first = true;
        if (kk & 1) {
          load_chain_op<AQ>(M1, acl4, kk, lane);
          hop(kk, true, T_{});
          first = false;
          --kk;
        } else {
          load_chain_op<AQ>(M0, acl4, kk, lane);
        }
        for (; kk >= 2; kk -= 2) {
          hop(kk, first, F_{});
          first = false;
          hop(kk - 1, false, T_{});
        }
        if (first) flag_wait(sync + kSyncG, N, T, sync + kSyncAbort, lane);  // N == 1: no hop waited
        // k = 0: p'_0 only
        if (lb == 0) lds_store<RB>(ppf + la * RB, pv);
        flag_set(sync + kSyncP, T);
#pragma unroll
        for (int i = 0; i < RB; ++i) p0[i] = pv[i];
      }
      // forward chain, k = 0 .. N-1: xt_{k+1} = A_cl,k xt_k + e_k, stored and
      // flagged; the relaxed x_N and p_N for the next iteration come from xt_N
      // before the last flag lets stage N-1 overwrite x_N
      {
        float xv[RB];  // xt_k of the coming hop, in its input layout
        // Hop kk, prefetching stage `next` (none if negative).  ODD: xt_k on
        // a*RB + j, summed over a, xt_{k+1} on b*RB + i; even: roles swap.
        auto hop = [&](int kk, int next, auto odd_c) {
          constexpr bool ODD = decltype(odd_c)::value;
          const int out_idx = ODD ? lb * RB : la * RB;
          int ok = kk * NXP;
          opaque_s(ok);
          float ev[RB], sx[RB];
          lds_load<RB>(ev, ef + ok + out_idx);
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = 0.f;
          if constexpr (ODD) {
            if (next >= 0) load_chain_op<AQ>(M0, acl4, next, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
              for (int i = 0; i < RB; ++i) sx[i] += M1[i * RB + j] * xv[j];
            red_a_all<RB>(sx);
          } else {
            load_chain_op<AQ>(M1, acl4, next, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
              for (int i = 0; i < RB; ++i) sx[i] += M0[i * RB + j] * xv[j];
#pragma unroll
            for (int i = 0; i < RB; ++i) sx[i] = red_b(sx[i]);
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) xv[i] = ev[i] + sx[i];
          if ((ODD ? la : lb) == 0) lds_store<RB>(xtf + ok + NXP + out_idx, xv);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        // stage 0: xt_1 = A_cl,0 x_0 + g'_0 + S_0 p'_0, without waiting for C_0;
        // the wait for e_1 .. e_{N-1} comes after xt_1 is out
        if (N > 1) load_chain_op<AQ>(M1, acl4, 1, lane);
        {
          // S_0 (in M0) acts in the even stages' form, which sums over b: p'_0
          // moves from a*RB + j to b*RB + j first (lane (a, b) reads lane (b, a))
          float g0[RB], pt[RB], sx[RB];
          const int src = ((lb << 3) | la) << 2;
#pragma unroll
          for (int j = 0; j < RB; ++j)
            pt[j] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p0[j])));
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = 0.f;
#pragma unroll
          for (int j = 0; j < RB; ++j)
#pragma unroll
            for (int i = 0; i < RB; ++i) sx[i] += M0[i * RB + j] * pt[j];
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = red_b(sx[i]);
          flag_wait(sync + kSyncE, 1, T, sync + kSyncAbort, lane);  // g'_0
          lds_load<RB>(g0, g0f + (T & 1) * NXP + la * RB);
#pragma unroll
          for (int i = 0; i < RB; ++i) xv[i] = ax0[i] + g0[i] + sx[i];
        }
        if (lb == 0) lds_store<RB>(xtf + NXP + la * RB, xv);
        if (N > 1) flag_set(sync + kSyncX + 1, T);
        // e_k of stages k >= 1; x_N as relaxed in the previous iteration
        // (stage N-1 wrote it before flagging)
        if (N > 1) flag_wait(sync + kSyncE + 1, N - 1, T, sync + kSyncAbort, lane);
        double xdN[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) xdN[i] = xd[N * NXP + pidx + i];
        int kk = 1;
        for (; kk + 1 < N; kk += 2) {
          hop(kk, kk + 1, T_{});
          flag_set(sync + kSyncX + kk + 1, T);
          // the last pair prefetches stage N-1 again rather than branch
          hop(kk + 1, kk + 2 < N ? kk + 2 : N - 1, F_{});
          if (kk + 2 < N) flag_set(sync + kSyncX + kk + 2, T);
        }
        if (kk < N) hop(kk, -1, T_{});
        // xt_N is in xv now, in the layout pidx; x_N (the previous iteration's
        // relaxation, which stage N-1 overwrites once xt_N is flagged) was read
        // at the start of the chain
        flag_set(sync + kSyncX + N, T);
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const double xn = alpha * (double)xv[i] + oma * xdN[i];
          pN[i] = (float)(-(qd[pidx + i] * xrd[N * NXP + pidx + i]) - sigma * xn);
        }
      }
    }
  } else {
    // ---------------- stage wavefront k ----------------
    // (a launch may be wider than this agent: wavefronts past its chain
    // wavefront idle, joining only the workgroup barriers)
    float Km[CB][RB], Bm[RB][CB], Hm[CB][CB];
    {
      const bool own = w < N;
      const float* src = fws + d.ofw + ((int64_t)w * SLOTS + 4 * AQ) * 64 + lane;
#pragma unroll
      for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) Km[i][j] = own ? src[(i * RB + j) * 64] : 0.f;
      src += CB * RB * 64;
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) Bm[i][j] = own ? src[(i * CB + j) * 64] : 0.f;
      src += RB * CB * 64;
#pragma unroll
      for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) Hm[i][j] = own ? src[(i * CB + j) * 64] : 0.f;
    }
    // x^0 rollout: this stage's B_k (u_k - K_k x_k) + c_k when the chain reaches it
    for (int kk = 0; kk < N; ++kk) {
      if (w == kk) {
        float xa[RB], v[CB];
#pragma unroll
        for (int j = 0; j < RB; ++j) xa[j] = (float)xd[kk * NXP + la * RB + j];
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < RB; ++j) s += (double)(Km[i][j] * xa[j]);
          v[i] = (float)(ud[kk * NUP + lb * CB + i] - red_a(s));
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < CB; ++j) s += (double)(Bm[i][j] * v[j]);
          s = red_b(s);
          const int idx = la * RB + i;
          if (lb == 0 && idx < NX) bvd[idx] = (double)cf[kk * NXP + idx] + s;
        }
      }
      __syncthreads();
      __syncthreads();
    }
    // x_N <- alpha xt_N + (1 - alpha) x_N once the forward chain of iteration t is out
    auto relax_xN = [&](int t) {
      flag_wait(sync + kSyncX + N, 1, t, sync + kSyncAbort, lane);
      for (int i = lane; i < NX; i += 64)
        xd[N * NXP + i] = alpha * (double)xtf[N * NXP + i] + oma * xd[N * NXP + i];
    };
    // Per-lane row bookkeeping of this stage, fixed for the solve.  Row i < M:
    // (C u)_i = zc_s1 u[zc_i1] + zc_s2 u[zc_i2].  Input j < NU: (C' w)_j = w_j
    // plus, for a foot's pyramid components, its four pyramid rows from rt_b0
    // (rt_cc picks the combination; other components add nothing).
    int zc_i1 = 0, zc_i2 = 0, rt_b0 = 0, rt_cc = -1;
    double zc_s1 = 0.0, zc_s2 = 0.0, u_own = 0.0, ru_own = 0.0;
    if (lane < M) {
      if (lane < NU) {
        zc_i1 = zc_i2 = lane;
        zc_s1 = 1.0;
      } else {
        const int f = (lane - NU) >> 2, pp = (lane - NU) & 3, b = d.n_tau + f * d.foot_dim;
        zc_i1 = pp < 2 ? b : b + 1;
        zc_s1 = (pp & 1) ? -1.0 : 1.0;
        zc_i2 = b + 2;
        zc_s2 = -mu;
      }
    }
    if (lane < NU && lane >= d.n_tau) {
      rt_b0 = NU + 4 * ((lane - d.n_tau) / d.foot_dim);
      rt_cc = (lane - d.n_tau) % d.foot_dim;
    }
    // The no-slip rows' terms of stage k's state weight (k >= 1), entry i:
    // Jc' w_c,k, and on the last stage also (Jc A_cl,N-1)' w_c,N, through which
    // the rows of x_N reach p_{N-1}; the last stage leaves Jc' w_c,N for its C
    // (p'_{N-1} = p_N + s_{N-1}, p_N holding Jc' w_c,N).
    // Rows in blocks of 4, every LDS load of a block issued before the first
    // add (rows past nc clamped and not added), so that the loads do not wait
    // one by one on the last stage's critical path.
    auto row_terms = [&](int i) -> double {
      double v = 0.0;
      for (int r0 = 0; r0 < nc; r0 += 4) {
        float jv[4];
        double wv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rw = min(r0 + t, nc - 1);
          jv[t] = jc[rw * NXP + i];
          wv[t] = wcd[(k - 1) * nc + rw];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (r0 + t < nc) v += (double)jv[t] * wv[t];
      }
      if (k == N - 1) {
        double dn = 0.0;
        for (int r0 = 0; r0 < nc; r0 += 4) {
          float av[4], jv[4];
          double wn[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int rw = min(r0 + t, nc - 1);
            av[t] = jac[rw * NXP + i];
            jv[t] = jc[rw * NXP + i];
            wn[t] = wcd[(N - 1) * nc + rw];
          }
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (r0 + t < nc) {
              v += (double)av[t] * wn[t];
              dn += (double)jv[t] * wn[t];
            }
        }
        dnf[i] = (float)dn;
      }
      return v;
    };
    if (k < N) {
      if (lane < NU) {
        u_own = ud[k * NUP + lane];
        if (uref) ru_own = (double)r[lane] * (double)uref[(int64_t)k * NU + lane];
      }
      if (lane < M) wvd[k * M + lane] = yd[k * M + lane] - rhod[k * M + lane] * zd[k * M + lane];
      if (k >= 1 && lane < NX)
        qtd[k * NXP + lane] = -qd[lane] * xrd[k * NXP + lane] - sigma * xd[k * NXP + lane] + (nc ? row_terms(lane) : 0.0);
      wave_sync();
    }
    const int n_it = w < N ? iters : 0;  // wavefronts past the chain wavefront idle
    for (int it = 0; it < n_it; ++it) {
      const int T = it + 1;
      // (A) linear terms of stage k: rt_k, g_k = qt_k + K_k' rt_k
      if (w < N) {
        // rt_k = C_k'(y_k - rho_k z_k) - sigma u_k - R ubar_k, from the row
        // terms w = y - rho z that E left in LDS (lane j < NU: its own row and
        // the four pyramid rows of its foot)
        if (lane < NUP) {
          double v = 0.0;
          if (lane < NU) {
            const double* wk = wvd + k * M;
            const double w0 = wk[rt_b0], w1 = wk[rt_b0 + 1], w2 = wk[rt_b0 + 2], w3 = wk[rt_b0 + 3];
            v = wk[lane];
            if (rt_cc == 0) v += w0 - w1;
            if (rt_cc == 1) v += w2 - w3;
            if (rt_cc == 2) v -= mu * (w0 + w1 + w2 + w3);
            v += -sigma * u_own;
            v -= ru_own;
          }
          rtd[k * NUP + lane] = v;
        }
        wave_sync();
        // Every product below forms all its partial sums first, then all its
        // butterflies, then one guarded store, so the independent chains
        // interleave instead of serialising behind the store's branch.
        if (k >= 1) {
          float rv[CB], sg[RB];
          double qt[RB];
#pragma unroll
          for (int i = 0; i < CB; ++i) rv[i] = (float)rtd[k * NUP + lb * CB + i];
#pragma unroll
          for (int j = 0; j < RB; ++j) qt[j] = qtd[k * NXP + la * RB + j];
#pragma unroll
          for (int j = 0; j < RB; ++j) sg[j] = 0.f;
#pragma unroll
          for (int i = 0; i < CB; ++i)
#pragma unroll
            for (int j = 0; j < RB; ++j) sg[j] += Km[i][j] * rv[i];
#pragma unroll
          for (int j = 0; j < RB; ++j) sg[j] = red_b(sg[j]);
          if (lb == 0)
#pragma unroll
            for (int j = 0; j < RB; ++j) {
              const int idx = la * RB + j;
              gf[k * NXP + idx] = (float)(qt[j] + (double)sg[j]);
            }
        }
      }
      flag_set(sync + kSyncG + k, T);
      // The relaxed x_N of the previous iteration (nothing else in this
      // iteration needs it before the forward chain reads it again); the chain
      // wavefront has taken its own copy for p_N before flagging xt_N.
      if (k == N - 1 && it >= 1) relax_xN(T - 1);
      if (k == 0) {
        // g'_0 = c_0 - B_0 H_0^{-1} rt_0, the part of xt_1 that does not depend
        // on p'_0 (the chain wavefront adds S_0 p'_0); flagged as stage 0's e
        // (after the relaxation of x_N when stage 0 is the last).  dd_0 holds
        // -H_0^{-1} rt_0 until C_0 overwrites it with d_0.
        float hv[CB], sd[CB], dv[CB], se[RB];
#pragma unroll
        for (int j = 0; j < CB; ++j) hv[j] = (float)rtd[lb * CB + j];
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] = 0.f;
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int i = 0; i < CB; ++i) sd[i] += Hm[i][j] * hv[j];
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] = red_b(sd[i]);
        if (lb == 0)
#pragma unroll
          for (int i = 0; i < CB; ++i) dd[la * CB + i] = -(double)sd[i];
        wave_sync();
#pragma unroll
        for (int j = 0; j < CB; ++j) dv[j] = (float)dd[lb * CB + j];
#pragma unroll
        for (int i = 0; i < RB; ++i) se[i] = 0.f;
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int i = 0; i < RB; ++i) se[i] += Bm[i][j] * dv[j];
#pragma unroll
        for (int i = 0; i < RB; ++i) se[i] = red_b(se[i]);
        if (lb == 0)
#pragma unroll
          for (int i = 0; i < RB; ++i) g0f[(T & 1) * NXP + la * RB + i] = cf[la * RB + i] + se[i];
        flag_set(sync + kSyncE, T);
      }
      // (B) backward chain on the chain wavefront; C_k starts once p'_k is out
      flag_wait(sync + kSyncP + k, 1, T, sync + kSyncAbort, lane);
      // (C) d_k = -H_k^{-1}(rt_k + B_k' p'_k), e_k = B_k d_k + c_k
      if (w < N) {
        float pv[RB], hv[CB], sh[CB], sd[CB];
        double rtv[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) pv[i] = ppf[k * NXP + la * RB + i];
        if (nc && k == N - 1)
#pragma unroll
          for (int i = 0; i < RB; ++i) pv[i] += dnf[la * RB + i];
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          rtv[j] = rtd[k * NUP + lb * CB + j];
          sh[j] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j) sh[j] += Bm[i][j] * pv[i];
        red_a_all<CB>(sh);
#pragma unroll
        for (int j = 0; j < CB; ++j) hv[j] = (float)(rtv[j] + (double)sh[j]);
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] = 0.f;
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int i = 0; i < CB; ++i) sd[i] += Hm[i][j] * hv[j];
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] = red_b(sd[i]);
        if (lb == 0)
#pragma unroll
          for (int i = 0; i < CB; ++i) dd[k * NUP + la * CB + i] = -(double)sd[i];
        wave_sync();
      }
      if (w < N && k >= 1) {  // stage 0's part of xt_1 is g'_0 + S_0 p'_0
        float dv[CB], cv[RB], se[RB];
#pragma unroll
        for (int j = 0; j < CB; ++j) dv[j] = (float)dd[k * NUP + lb * CB + j];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          cv[i] = cf[k * NXP + la * RB + i];
          se[i] = 0.f;
        }
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int i = 0; i < RB; ++i) se[i] += Bm[i][j] * dv[j];
#pragma unroll
        for (int i = 0; i < RB; ++i) se[i] = red_b(se[i]);
        if (lb == 0)
#pragma unroll
          for (int i = 0; i < RB; ++i) ef[k * NXP + la * RB + i] = cv[i] + se[i];
      }
      if (k >= 1) flag_set(sync + kSyncE + k, T);  // stage 0 flagged g'_0 before its C
      // (D) forward chain on the chain wavefront; E_k starts once xt_k is out
      if (k >= 1) flag_wait(sync + kSyncX + k, 1, T, sync + kSyncAbort, lane);
      // (E) ut_k = K_k xt_k + d_k; relaxation, projection and dual update of stage k
      if (w < N && nc) {
        // no-slip rows: zeta = Jc xt_k (k >= 1), and on the last stage the rows of
        // x_N, zeta = (Jc A_cl,N-1) xt_{N-1} + Jc e_{N-1}; relaxed, projected
        // (stance rows to 0, free rows to w + y_c / rho_c), dual update.  Quad
        // rw of the wavefront sums row r0 + rw, each lane every fourth column.
        const int part = lane & 3;
        auto row_update = [&](int kr, int rw, double zeta) {
          const int idx = (kr - 1) * nc + rw;
          const double rs = rcd[idx], rr = fabs(rs);
          const bool eq = rs < 0.0;
          const double wv = alpha * zeta + oma * zcd[idx];
          const double zn = eq ? 0.0 : wv + ycd[idx] * ircd[idx];
          const double yn = ycd[idx] + rr * (wv - zn);
          ycd[idx] = yn;
          zcd[idx] = zn;
          wcd[idx] = yn - rr * zn;
        };
        for (int r0 = 0; r0 < nc; r0 += 16) {
          const int rw = r0 + (lane >> 2);
          const int rc = min(rw, nc - 1);  // lanes past the last row read it and discard the sum
          constexpr int TQ = (NX + 3) / 4;  // columns per lane, read four at a time
          // sum over this lane's columns of u[col] * v[col], four loads of each in flight
          auto dot4 = [&](const float* u, const float* v) -> double {
            double acc = 0.0;
#pragma unroll
            for (int t0 = 0; t0 < TQ; t0 += 4) {
              float uv[4], vv[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int i = min(part + 4 * (t0 + t), NX - 1);
                uv[t] = u[i];
                vv[t] = v[i];
              }
#pragma unroll
              for (int t = 0; t < 4; ++t)
                if (t0 + t < TQ && part + 4 * (t0 + t) < NX) acc += (double)uv[t] * (double)vv[t];
            }
            return acc;
          };
          if (k >= 1) {
            double zeta = dot4(jc + rc * NXP, xtf + k * NXP);
            zeta = quad_sum(zeta);
            if (rw < nc && part == 0) row_update(k, rw, zeta);
          }
          if (k == N - 1) {
            // (Jc A_cl,N-1) xt_{N-1}, then Jc e_{N-1}
            double zeta = dot4(jac + rc * NXP, xtf + k * NXP);
            zeta += dot4(jc + rc * NXP, ef + k * NXP);
            zeta = quad_sum(zeta);
            if (rw < nc && part == 0) row_update(N, rw, zeta);
          }
        }
      }
      if (w < N) {
        float xv[RB], su[CB];
        double dvv[CB];
#pragma unroll
        for (int j = 0; j < RB; ++j) xv[j] = xtf[k * NXP + la * RB + j];
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          dvv[i] = dd[k * NUP + lb * CB + i];
          su[i] = 0.f;
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
          for (int i = 0; i < CB; ++i) su[i] += Km[i][j] * xv[j];
        red_a_all<CB>(su);
        if (la == 0)
#pragma unroll
          for (int i = 0; i < CB; ++i) utd[k * NUP + lb * CB + i] = dvv[i] + (double)su[i];
        wave_sync();
        // relaxed x_k and its qt_k = -Q x_ref,k - sigma x_k for the next A
        if (k >= 1 && lane < NX) {
          const double xn = alpha * (double)xtf[k * NXP + lane] + oma * xd[k * NXP + lane];
          xd[k * NXP + lane] = xn;
          qtd[k * NXP + lane] = -qd[lane] * xrd[k * NXP + lane] - sigma * xn + (nc ? row_terms(lane) : 0.0);
        }
        // row `lane`: (C ut)_i, relaxation, projection, dual update, w = y - rho z
        if (lane < M) {
          const int idx = k * M + lane;
          const double zeta = zc_s1 * utd[k * NUP + zc_i1] + zc_s2 * utd[k * NUP + zc_i2];
          const double wv = alpha * zeta + oma * zd[idx];
          const double zn = fmin(fmax(wv + yd[idx] * irhod[idx], lod[idx]), hid[idx]);
          const double yn = yd[idx] + rhod[idx] * (wv - zn);
          yd[idx] = yn;
          zd[idx] = zn;
          wvd[idx] = yn - rhod[idx] * zn;
        }
        if (lane < NU) {
          u_own = alpha * utd[k * NUP + lane] + oma * u_own;
          ud[k * NUP + lane] = u_own;
        }
        wave_sync();
      }
    }
    if (k == N - 1 && n_it > 0) relax_xN(n_it);
  }
  __syncthreads();

  bool fin = true;
  for (int i = tid; i < (N + 1) * NX; i += nt) {
    const float v = (float)xd[(i / NX) * NXP + i % NX];
    X[i] = v;
    fin &= (bool)isfinite(v);
  }
  for (int i = tid; i < N * NU; i += nt) {
    const float v = (float)ud[(i / NU) * NUP + i % NU];
    U[i] = v;
    fin &= (bool)isfinite(v);
  }
  for (int i = tid; i < N * M; i += nt) {
    Z[i] = (float)zd[i];
    Y[i] = (float)yd[i];
    fin &= (bool)isfinite(Z[i]) && (bool)isfinite(Y[i]);
  }
  for (int i = tid; i < N * nc; i += nt) {
    st.zc[d.ozc + i] = (float)zcd[i];
    st.yc[d.ozc + i] = (float)ycd[i];
    fin &= (bool)isfinite(zcd[i]) && (bool)isfinite(ycd[i]);
  }
  if (!fin || sync[kSyncAbort]) atomicOr(flag, 1);
  __syncthreads();
  if (tid == 0 && flag[0]) st.status[agent] = AGENT_NONFINITE;
}

// ------------------------------------------------------------------------------------
// ADMM iterations for longer horizons (kMaxStages <= N <= kMaxStream): the same
// split into stage wavefronts and one chain wavefront, with A_cl streamed from
// HBM through an LDS ring by a loader wavefront
// ------------------------------------------------------------------------------------

constexpr int kMaxStream = 20;  // longest horizon of the streaming iteration kernel
constexpr int kRing = 4;        // A_cl slots of its LDS ring
// flags: g_k, p'_k, e_k, xt_k ready (as kSync*), the ring slots' element numbers,
// the chain's consumed-element count, abort
constexpr int kStG = 0, kStP = kMaxStream + 1, kStE = 2 * (kMaxStream + 1), kStX = 3 * (kMaxStream + 1);
constexpr int kStRing = 4 * (kMaxStream + 1), kStUsed = kStRing + kRing, kStAbort = kStUsed + 1;
constexpr int kStInts = kStAbort + 1;

struct StreamLds {
  int ring, s0, xtf, ppf, gf, ef, sf, cf, g0f;                            // float
  int xd, ud, zd, yd, lod, hid, rhod, irhod, wvd, rtd, dd, utd, qd, xrd, qtd;  // double
  int flag, sync, total;
};

template <int NX, int NU>
__host__ __device__ inline StreamLds stream_lds_layout(int N, int M) {
  using S = FS<NX, NU>;
  StreamLds L{};
  int o = 0;
  auto take = [&](int bytes) {
    const int r = o;
    o += (bytes + 15) & ~15;
    return r;
  };
  L.ring = take(4 * kRing * S::AQ * 256);
  L.s0 = take(4 * S::AQ * 256);
  L.xtf = take(4 * (N + 1) * S::NXP);
  L.ppf = take(4 * N * S::NXP);
  L.gf = take(4 * N * S::NXP);
  L.ef = take(4 * N * S::NXP);
  L.sf = take(4 * N * S::NXP);
  L.cf = take(4 * N * S::NXP);
  L.g0f = take(4 * 2 * S::NXP);
  L.xd = take(8 * (N + 1) * S::NXP);
  L.ud = take(8 * N * S::NUP);
  L.zd = take(8 * N * M);
  L.yd = take(8 * N * M);
  L.lod = take(8 * N * M);
  L.hid = take(8 * N * M);
  L.rhod = take(8 * N * M);
  L.irhod = take(8 * N * M);
  L.wvd = take(8 * N * M);
  L.rtd = take(8 * N * S::NUP);
  L.dd = take(8 * N * S::NUP);
  L.utd = take(8 * N * S::NUP);
  L.qd = take(8 * S::NXP);
  L.xrd = take(8 * (N + 1) * S::NXP);
  L.qtd = take(8 * N * S::NXP);
  L.flag = take(16);
  L.sync = take(4 * kStInts);
  L.total = o;
  return L;
}

// The chain wavefront's operator sequence: stages 0 (for the constant
// A_cl,0 x_0), N-1 and N-2, then every iteration the backward chain's
// N-3 .. 1 and the forward chain's 3 .. N-1.  The two operators a chain ends
// on are the two the other chain starts with, still in registers, and A_cl,0
// is not needed again.  N >= 4.
__host__ __device__ inline int stream_stage(int g, int N) {
  if (g < 3) return g == 0 ? 0 : N - g;
  const int r = (g - 3) % (2 * N - 6);
  return r < N - 3 ? N - 3 - r : r - N + 6;
}
__host__ __device__ inline int stream_elements(int N, int iters) { return 3 + iters * (2 * N - 6); }

// Stage wavefront j owns stages j and j + SW (SW = ceil(N/2)) with K, B in
// registers and H^{-1} read from HBM before each C; the chain wavefront (SW)
// is the register-resident kernel's, taking A_cl,k from the ring; the loader
// wavefront (SW + 1) keeps three ring elements in flight.
template <int NX, int NU>
__device__ __forceinline__ void admm_stream_agent(const AgentDesc* __restrict__ desc, int agent,
                                                  Inputs<float> in, SolverConsts sc_all, int iters,
                                                  int warm, const float* __restrict__ fws,
                                                  State<float> st) {
  using S = FS<NX, NU>;
  constexpr int RB = S::RB, CB = S::CB, NXP = S::NXP, NUP = S::NUP, SLOTS = S::SLOTS, AQ = S::AQ;
  const SolverConsts sc = agent_consts(sc_all, agent);
  const AgentDesc d = desc[agent];
  const int N = d.N, M = d.m;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = tid >> 6, lane = tid & 63, la = lane >> 3, lb = lane & 7;
  float* X = st.x + d.ox;
  float* U = st.u + d.ou;
  float* Z = st.z + d.oz;
  float* Y = st.y + d.oy;
  if (st.status[agent] != AGENT_OK) {
    for (int i = tid; i < (N + 1) * d.nx; i += nt) X[i] = NAN;
    for (int i = tid; i < N * d.nu; i += nt) U[i] = NAN;
    for (int i = tid; i < N * M; i += nt) {
      Z[i] = NAN;
      Y[i] = NAN;
    }
    return;
  }
  const StreamLds L = stream_lds_layout<NX, NU>(N, M);
  extern __shared__ __align__(16) unsigned char sm[];
  float4* ring4 = reinterpret_cast<float4*>(sm + L.ring);
  float* xtf = reinterpret_cast<float*>(sm + L.xtf);
  float* ppf = reinterpret_cast<float*>(sm + L.ppf);
  float* gf = reinterpret_cast<float*>(sm + L.gf);
  float* ef = reinterpret_cast<float*>(sm + L.ef);
  float* sf = reinterpret_cast<float*>(sm + L.sf);
  float* cf = reinterpret_cast<float*>(sm + L.cf);
  float* g0f = reinterpret_cast<float*>(sm + L.g0f);  // g'_0 of iterations of odd / even number
  double* xd = reinterpret_cast<double*>(sm + L.xd);
  double* ud = reinterpret_cast<double*>(sm + L.ud);
  double* zd = reinterpret_cast<double*>(sm + L.zd);
  double* yd = reinterpret_cast<double*>(sm + L.yd);
  double* lod = reinterpret_cast<double*>(sm + L.lod);
  double* hid = reinterpret_cast<double*>(sm + L.hid);
  double* rhod = reinterpret_cast<double*>(sm + L.rhod);
  double* irhod = reinterpret_cast<double*>(sm + L.irhod);
  double* wvd = reinterpret_cast<double*>(sm + L.wvd);
  double* rtd = reinterpret_cast<double*>(sm + L.rtd);
  double* dd = reinterpret_cast<double*>(sm + L.dd);
  double* utd = reinterpret_cast<double*>(sm + L.utd);
  double* qd = reinterpret_cast<double*>(sm + L.qd);
  double* xrd = reinterpret_cast<double*>(sm + L.xrd);
  double* qtd = reinterpret_cast<double*>(sm + L.qtd);
  int* flag = reinterpret_cast<int*>(sm + L.flag);
  int* sync = reinterpret_cast<int*>(sm + L.sync);
  int* abortp = sync + kStAbort;

  const float* A = in.A + d.oA;
  const float* B = in.B + d.oB;
  const float* c = in.c + d.oc;
  const float* q = in.q + d.oq;
  const float* r = in.r + d.orr;
  const float* xr = in.xr + d.oxr;
  const float* x0 = in.x0 + d.ox0;
  const float* tau = in.tau + d.otau;
  const uint8_t* stance = in.st + d.ost;
  const float* uref = in.uref ? in.uref + d.our : nullptr;
  const double mu = (double)in.mu[d.omu];
  const float* opg = fws + d.ofw;  // this agent's operators in HBM

  // per-agent vectors into LDS (padding zero)
  for (int i = tid; i < L.total / 4; i += nt) reinterpret_cast<int*>(sm)[i] = 0;
  __syncthreads();
  {
    // S_0 from the factor (after the stage slots and s_k) into its LDS slot
    const float4* src = reinterpret_cast<const float4*>(opg + (int64_t)N * (SLOTS * 64 + NXP));
    float4* dst = reinterpret_cast<float4*>(sm + L.s0);
    for (int i = tid; i < AQ * 64; i += nt) dst[i] = src[i];
  }
  const float* sk = opg + (int64_t)N * SLOTS * 64;
  for (int i = tid; i < N * NXP; i += nt) sf[i] = sk[i];
  for (int i = tid; i < N * NX; i += nt) cf[(i / NX) * NXP + i % NX] = c[i];
  for (int i = tid; i < NX; i += nt) {
    qd[i] = (double)q[i];
    xd[i] = (double)x0[i];
    xtf[i] = x0[i];
  }
  for (int i = tid; i < (N + 1) * NX; i += nt) xrd[(i / NX) * NXP + i % NX] = (double)xr[i];
  for (int i = tid; i < N * M; i += nt) {
    const int k = i / M, j = i % M;
    double lo, hi, rr;
    row_bounds<double, float>(d, j, stance + k * d.n_feet, tau, sc, lo, hi, rr);
    lod[i] = lo;
    hid[i] = hi;
    rhod[i] = rr;
    irhod[i] = 1.0 / rr;
  }
  const bool wm = agent_warm(warm, d);
  for (int i = tid; i < N * NU; i += nt) ud[(i / NU) * NUP + i % NU] = wm ? (double)U[i] : 0.0;
  for (int i = tid; i < N * M; i += nt) {
    zd[i] = wm ? (double)Z[i] : 0.0;
    yd[i] = wm ? (double)Y[i] : 0.0;
  }
  __syncthreads();
  rollout_exact<NX, NU>(A, B, c, xd, ud, N, tid, nt);

  const double sigma = sc.sigma, alpha = sc.alpha, oma = 1.0 - sc.alpha;
  const int SW = (N + 1) / 2;  // stage wavefronts

  if (w == SW) {
    // ---------------- chain wavefront ----------------
    __builtin_amdgcn_s_setprio(2);
    float M0[4 * AQ], M1[4 * AQ];  // even / odd stage operators
    // S_0 = -B_0 H_0^{-1} B_0' in LDS (xt_1 = A_cl,0 x_0 + g'_0 + S_0 p'_0)
    const float4* s04 = reinterpret_cast<const float4*>(sm + L.s0);
    int e = 0;                     // next element of the operator sequence
    int el0 = 0, el1 = 0;          // elements held in M0 / M1
    int seen0 = 0, seen1 = 0;      // their slot's flag as read with them
    // Element e from the ring, read speculatively: the slot's flag first, then
    // the operator (this wavefront's LDS reads complete in issue order, so the
    // operator is the published one whenever the flag already was).
    auto fetch = [&](float (&Mx)[4 * AQ], int& elx, int& seenx) __attribute__((always_inline)) {
      const int slot = e & (kRing - 1);
      seenx = __hip_atomic_load(sync + kStRing + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      asm volatile("" ::: "memory");
      load_chain_op<AQ>(Mx, ring4, slot, lane);
      elx = e++;
    };
    // Before an operator's first use: reread it if its flag was not yet set,
    // then hand its slot back to the loader.
    auto settle = [&](float (&Mx)[4 * AQ], int elx, int seenx) __attribute__((always_inline)) {
      if (!__all(seenx >= elx + 1)) {
        flag_wait(sync + kStRing + (elx & (kRing - 1)), 1, elx + 1, abortp, lane);
        load_chain_op<AQ>(Mx, ring4, elx & (kRing - 1), lane);
      }
      flag_set(sync + kStUsed, elx + 1);
    };
    const int pidx = ((N - 1) & 1) ? lb * RB : la * RB;
    float pN[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
      pN[i] = (float)(-qd[pidx + i] * xrd[N * NXP + pidx + i] - sigma * xd[N * NXP + pidx + i]);
    float ax0[RB];
    {
      fetch(M0, el0, seen0);  // stage 0
      settle(M0, el0, seen0);
      float x0v[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) x0v[j] = xtf[lb * RB + j];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        ax0[i] = 0.f;
#pragma unroll
        for (int j = 0; j < RB; ++j) ax0[i] += M0[i * RB + j] * x0v[j];
        ax0[i] = red_b(ax0[i]);
      }
    }
    // stages N-1 and N-2, the backward chain's first operators
    for (int kk = N - 1; kk >= N - 2; --kk) {
      if (kk & 1) {
        fetch(M1, el1, seen1);
        settle(M1, el1, seen1);
      } else {
        fetch(M0, el0, seen0);
        settle(M0, el0, seen0);
      }
    }
    using T_ = std::true_type;
    using F_ = std::false_type;
    float p0[RB];  // p'_0 of the current iteration, on a*RB + i
    for (int it = 0; it < iters; ++it) {
      const int T = it + 1;
      {
        float pv[RB];
        // hop kk of the backward chain: its operator is settled here unless it
        // is stage N-1 or N-2 (already in registers); fetches stage kk-1 for
        // 2 <= kk <= N-2
        auto hop = [&](int kk, bool first, auto odd_c) __attribute__((always_inline)) {
          constexpr bool ODD = decltype(odd_c)::value;
          const int in_idx = ODD ? lb * RB : la * RB, out_idx = ODD ? la * RB : lb * RB;
          if (kk <= N - 3) {
            if constexpr (ODD) settle(M1, el1, seen1);
            else settle(M0, el0, seen0);
          }
          int ok = kk * NXP, om = (kk - 1) * NXP;
          opaque_s(ok);
          opaque_s(om);
          if ((ODD ? la : lb) == 0) lds_store<RB>(ppf + ok + in_idx, pv);
          flag_set(sync + kStP + kk, T);  // C_kk may start now
          float gv[RB], sv[RB], qv[RB];
          lds_load<RB>(sv, sf + om + out_idx);
          lds_load<RB>(gv, gf + ok + out_idx);
#pragma unroll
          for (int j = 0; j < RB; ++j) qv[j] = 0.f;
          if constexpr (ODD) {
            if (kk >= 2 && kk <= N - 2) fetch(M0, el0, seen0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
              for (int j = 0; j < RB; ++j) qv[j] += M1[i * RB + j] * pv[i];
#pragma unroll
            for (int j = 0; j < RB; ++j) qv[j] = red_b(qv[j]);
          } else {
            if (kk <= N - 2) fetch(M1, el1, seen1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
              for (int j = 0; j < RB; ++j) qv[j] += M0[i * RB + j] * pv[i];
            red_a_all<RB>(qv);
          }
          if (first) {
            flag_wait(sync + kStG, N, T, abortp, lane);
            lds_load<RB>(gv, gf + ok + out_idx);
          }
#pragma unroll
          for (int j = 0; j < RB; ++j) pv[j] = gv[j] + qv[j] + sv[j];
        };
        int kk = N - 1;
#pragma unroll
        for (int i = 0; i < RB; ++i) pv[i] = pN[i] + sf[kk * NXP + pidx + i];
        bool first = true;
        if (kk & 1) {
          hop(kk, true, T_{});
          first = false;
          --kk;
        }
        for (; kk >= 2; kk -= 2) {
          hop(kk, first, F_{});
          first = false;
          hop(kk - 1, false, T_{});
        }
        if (lb == 0) lds_store<RB>(ppf + la * RB, pv);
        flag_set(sync + kStP, T);
#pragma unroll
        for (int i = 0; i < RB; ++i) p0[i] = pv[i];
      }
      {
        float xv[RB];
        // hop kk of the forward chain: its operator is settled here unless it
        // is stage 1 or 2 (the backward chain's last two); fetches stage kk+1
        // for 2 <= kk <= N-2
        auto hop = [&](int kk, auto odd_c) __attribute__((always_inline)) {
          constexpr bool ODD = decltype(odd_c)::value;
          const int out_idx = ODD ? lb * RB : la * RB;
          if (kk >= 3) {
            if constexpr (ODD) settle(M1, el1, seen1);
            else settle(M0, el0, seen0);
          }
          int ok = kk * NXP;
          opaque_s(ok);
          float ev[RB], sx[RB];
          lds_load<RB>(ev, ef + ok + out_idx);
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = 0.f;
          if constexpr (ODD) {
            if (kk >= 2 && kk + 1 < N) fetch(M0, el0, seen0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
              for (int i = 0; i < RB; ++i) sx[i] += M1[i * RB + j] * xv[j];
            red_a_all<RB>(sx);
          } else {
            if (kk >= 2 && kk + 1 < N) fetch(M1, el1, seen1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
              for (int i = 0; i < RB; ++i) sx[i] += M0[i * RB + j] * xv[j];
#pragma unroll
            for (int i = 0; i < RB; ++i) sx[i] = red_b(sx[i]);
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) xv[i] = ev[i] + sx[i];
          if ((ODD ? la : lb) == 0) lds_store<RB>(xtf + ok + NXP + out_idx, xv);
        };
        // stage 0: xt_1 = A_cl,0 x_0 + g'_0 + S_0 p'_0, without waiting for
        // C_0; S_0 acts in the even stages' form (summed over b), so p'_0
        // moves from a*RB + j to b*RB + j first (lane (a, b) reads (b, a))
        {
          float g0[RB], pt[RB], sx[RB];
          const int src = ((lb << 3) | la) << 2;
#pragma unroll
          for (int j = 0; j < RB; ++j)
            pt[j] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p0[j])));
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = 0.f;
          // S_0 read from LDS three quads at a time: the chain keeps A_cl,1 and
          // A_cl,2 in registers across the turn, so S_0 gets no register set
#pragma unroll
          for (int q0 = 0; q0 < AQ; q0 += 3) {
            float4 v[3];
#pragma unroll
            for (int u = 0; u < 3; ++u)
              if (q0 + u < AQ) v[u] = s04[(q0 + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
              for (int c4 = 0; c4 < 4; ++c4) {
                const int e = 4 * (q0 + u) + c4;
                if (q0 + u < AQ && e < RB * RB) {
                  const float sv = c4 == 0 ? v[u].x : c4 == 1 ? v[u].y : c4 == 2 ? v[u].z : v[u].w;
                  sx[e / RB] += sv * pt[e % RB];
                }
              }
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) sx[i] = red_b(sx[i]);
          flag_wait(sync + kStE, 1, T, abortp, lane);  // g'_0
          lds_load<RB>(g0, g0f + (T & 1) * NXP + la * RB);
#pragma unroll
          for (int i = 0; i < RB; ++i) xv[i] = ax0[i] + g0[i] + sx[i];
        }
        if (lb == 0) lds_store<RB>(xtf + NXP + la * RB, xv);
        flag_set(sync + kStX + 1, T);
        // e_k of stages k >= 1; x_N as relaxed in the previous iteration
        // (the wavefront of stage N-1 wrote it before flagging e_{N-1})
        flag_wait(sync + kStE + 1, N - 1, T, abortp, lane);
        double xdN[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) xdN[i] = xd[N * NXP + pidx + i];
        int kk = 1;
        for (; kk + 1 < N; kk += 2) {
          hop(kk, T_{});
          flag_set(sync + kStX + kk + 1, T);
          hop(kk + 1, F_{});
          if (kk + 2 < N) flag_set(sync + kStX + kk + 2, T);
        }
        if (kk < N) hop(kk, T_{});
        flag_set(sync + kStX + N, T);
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const double xn = alpha * (double)xv[i] + oma * xdN[i];
          pN[i] = (float)(-(qd[pidx + i] * xrd[N * NXP + pidx + i]) - sigma * xn);
        }
      }
    }
  } else if (w == SW + 1) {
    // ---------------- loader wavefront ----------------
    // element g: global loads into a register set, then (once the chain has
    // handed back element g - kRing) into ring slot g % kRing and flagged;
    // three elements are in flight
    const int total = stream_elements(N, iters);
    const f4* src4 = reinterpret_cast<const f4*>(opg) + lane;
    f4 R[3][AQ];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const f4* src = src4 + (int64_t)stream_stage(j, N) * SLOTS * 16;
#pragma unroll
      for (int qv = 0; qv < AQ; ++qv) R[j][qv] = src[qv * 64];
    }
    for (int g0 = 0; g0 < total; g0 += 3) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int g = g0 + j;
        if (g < total) {
          if (g >= kRing) flag_wait(sync + kStUsed, 1, g - kRing + 1, abortp, lane);
          f4* dst = reinterpret_cast<f4*>(ring4) + (g & (kRing - 1)) * AQ * 64 + lane;
#pragma unroll
          for (int qv = 0; qv < AQ; ++qv) dst[qv * 64] = R[j][qv];
          flag_set(sync + kStRing + (g & (kRing - 1)), g + 1);
          if (g + 3 < total) {
            const f4* src = src4 + (int64_t)stream_stage(g + 3, N) * SLOTS * 16;
#pragma unroll
            for (int qv = 0; qv < AQ; ++qv) R[j][qv] = src[qv * 64];
          }
        }
      }
    }
  } else if (w < SW) {
    // ---------------- stage wavefront: stages w and w + SW ----------------
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int kS[2] = {wu, wu + SW};
    const bool hasH = kS[1] < N;
    float Km[2][CB][RB], Bm[2][RB][CB], Hm[CB][CB];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const bool own = kS[s2] < N;
      const float* src = opg + ((int64_t)(own ? kS[s2] : 0) * SLOTS + 4 * AQ) * 64 + lane;
#pragma unroll
      for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) Km[s2][i][j] = own ? src[(i * RB + j) * 64] : 0.f;
      src += CB * RB * 64;
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) Bm[s2][i][j] = own ? src[(i * CB + j) * 64] : 0.f;
    }
    auto load_H = [&](int k) __attribute__((always_inline)) {
      const float* src = opg + ((int64_t)k * SLOTS + 4 * AQ + 2 * CB * RB) * 64 + lane;
#pragma unroll
      for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) Hm[i][j] = src[(i * CB + j) * 64];
    };
    auto relax_xN = [&](int t) __attribute__((always_inline)) {
      flag_wait(sync + kStX + N, 1, t, abortp, lane);
      for (int i = lane; i < NX; i += 64)
        xd[N * NXP + i] = alpha * (double)xtf[N * NXP + i] + oma * xd[N * NXP + i];
    };
    int zc_i1 = 0, zc_i2 = 0, rt_b0 = 0, rt_cc = -1;
    double zc_s1 = 0.0, zc_s2 = 0.0;
    if (lane < M) {
      if (lane < NU) {
        zc_i1 = zc_i2 = lane;
        zc_s1 = 1.0;
      } else {
        const int f = (lane - NU) >> 2, pp = (lane - NU) & 3, b = d.n_tau + f * d.foot_dim;
        zc_i1 = pp < 2 ? b : b + 1;
        zc_s1 = (pp & 1) ? -1.0 : 1.0;
        zc_i2 = b + 2;
        zc_s2 = -mu;
      }
    }
    if (lane < NU && lane >= d.n_tau) {
      rt_b0 = NU + 4 * ((lane - d.n_tau) / d.foot_dim);
      rt_cc = (lane - d.n_tau) % d.foot_dim;
    }
    // (u_k stays in LDS, ud: register copies of it spill in this kernel)
    double ru_own[2] = {0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int k = kS[s2];
      if (k < N) {
        if (lane < NU && uref) ru_own[s2] = (double)r[lane] * (double)uref[(int64_t)k * NU + lane];
        if (lane < M) wvd[k * M + lane] = yd[k * M + lane] - rhod[k * M + lane] * zd[k * M + lane];
        if (k >= 1 && lane < NX) qtd[k * NXP + lane] = -qd[lane] * xrd[k * NXP + lane] - sigma * xd[k * NXP + lane];
      }
    }
    wave_sync();
    // (A) of stage kS[s]: rt_k and g_k = qt_k + K_k' rt_k, flagged for iteration t
    auto phaseA = [&](auto s_c, int t) __attribute__((always_inline)) {
      constexpr int s2 = decltype(s_c)::value;
      int k = kS[s2];
      opaque_s(k);  // per-stage addresses formed here, not kept live across the loop
      if (lane < NUP) {
        double v = 0.0;
        if (lane < NU) {
          const double* wk = wvd + k * M;
          const double w0 = wk[rt_b0], w1 = wk[rt_b0 + 1], w2 = wk[rt_b0 + 2], w3 = wk[rt_b0 + 3];
          v = wk[lane];
          if (rt_cc == 0) v += w0 - w1;
          if (rt_cc == 1) v += w2 - w3;
          if (rt_cc == 2) v -= mu * (w0 + w1 + w2 + w3);
          v += -sigma * ud[k * NUP + lane];
          v -= ru_own[s2];
        }
        rtd[k * NUP + lane] = v;
      }
      wave_sync();
      if (k >= 1) {
        float rv[CB], sg[RB];
        double qt[RB];
#pragma unroll
        for (int i = 0; i < CB; ++i) rv[i] = (float)rtd[k * NUP + lb * CB + i];
#pragma unroll
        for (int j = 0; j < RB; ++j) qt[j] = qtd[k * NXP + la * RB + j];
#pragma unroll
        for (int j = 0; j < RB; ++j) sg[j] = 0.f;
#pragma unroll
        for (int i = 0; i < CB; ++i)
#pragma unroll
          for (int j = 0; j < RB; ++j) sg[j] += Km[s2][i][j] * rv[i];
#pragma unroll
        for (int j = 0; j < RB; ++j) sg[j] = red_b(sg[j]);
        if (lb == 0)
#pragma unroll
          for (int j = 0; j < RB; ++j) gf[k * NXP + la * RB + j] = (float)(qt[j] + (double)sg[j]);
      }
      flag_set(sync + kStG + k, t);
    };
    // (C) of stage kS[s] (H^{-1} already in Hm)
    auto phaseC = [&](auto s_c, int t) __attribute__((always_inline)) {
      constexpr int s2 = decltype(s_c)::value;
      int k = kS[s2];
      opaque_s(k);  // per-stage addresses formed here, not kept live across the loop
      float pv[RB], hv[CB], sh[CB], sd[CB];
      double rtv[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) pv[i] = ppf[k * NXP + la * RB + i];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        rtv[j] = rtd[k * NUP + lb * CB + j];
        sh[j] = 0.f;
      }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) sh[j] += Bm[s2][i][j] * pv[i];
      red_a_all<CB>(sh);
#pragma unroll
      for (int j = 0; j < CB; ++j) hv[j] = (float)(rtv[j] + (double)sh[j]);
#pragma unroll
      for (int i = 0; i < CB; ++i) sd[i] = 0.f;
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] += Hm[i][j] * hv[j];
#pragma unroll
      for (int i = 0; i < CB; ++i) sd[i] = red_b(sd[i]);
      if (lb == 0)
#pragma unroll
        for (int i = 0; i < CB; ++i) dd[k * NUP + la * CB + i] = -(double)sd[i];
      wave_sync();
      float dv[CB], cv[RB], se[RB];
#pragma unroll
      for (int j = 0; j < CB; ++j) dv[j] = (float)dd[k * NUP + lb * CB + j];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        cv[i] = cf[k * NXP + la * RB + i];
        se[i] = 0.f;
      }
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int i = 0; i < RB; ++i) se[i] += Bm[s2][i][j] * dv[j];
#pragma unroll
      for (int i = 0; i < RB; ++i) se[i] = red_b(se[i]);
      // (stage 0's part of xt_1 is g'_0 + S_0 p'_0, formed by the chain)
      if (lb == 0 && k >= 1)
#pragma unroll
        for (int i = 0; i < RB; ++i) ef[k * NXP + la * RB + i] = cv[i] + se[i];
      if (k >= 1) flag_set(sync + kStE + k, t);
    };
    // g'_0 = c_0 - B_0 H_0^{-1} rt_0 of iteration t (stage 0's wavefront, H_0 in
    // Hm): the part of xt_1 that does not depend on p'_0, flagged as stage 0's
    // e.  dd_0 holds -H_0^{-1} rt_0 until C_0 overwrites it with d_0.
    auto gprime0 = [&](int t) __attribute__((always_inline)) {
      float hv[CB], sd[CB], dv[CB], se[RB];
#pragma unroll
      for (int j = 0; j < CB; ++j) hv[j] = (float)rtd[lb * CB + j];
#pragma unroll
      for (int i = 0; i < CB; ++i) sd[i] = 0.f;
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int i = 0; i < CB; ++i) sd[i] += Hm[i][j] * hv[j];
#pragma unroll
      for (int i = 0; i < CB; ++i) sd[i] = red_b(sd[i]);
      if (lb == 0)
#pragma unroll
        for (int i = 0; i < CB; ++i) dd[la * CB + i] = -(double)sd[i];
      wave_sync();
#pragma unroll
      for (int j = 0; j < CB; ++j) dv[j] = (float)dd[lb * CB + j];
#pragma unroll
      for (int i = 0; i < RB; ++i) se[i] = 0.f;
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int i = 0; i < RB; ++i) se[i] += Bm[0][i][j] * dv[j];
#pragma unroll
      for (int i = 0; i < RB; ++i) se[i] = red_b(se[i]);
      if (lb == 0)
#pragma unroll
        for (int i = 0; i < RB; ++i) g0f[(t & 1) * NXP + la * RB + i] = cf[la * RB + i] + se[i];
      flag_set(sync + kStE, t);
    };
    // (E) of stage kS[s]
    auto phaseE = [&](auto s_c) __attribute__((always_inline)) {
      constexpr int s2 = decltype(s_c)::value;
      int k = kS[s2];
      opaque_s(k);  // per-stage addresses formed here, not kept live across the loop
      float xv[RB], su[CB];
      double dvv[CB];
#pragma unroll
      for (int j = 0; j < RB; ++j) xv[j] = xtf[k * NXP + la * RB + j];
#pragma unroll
      for (int i = 0; i < CB; ++i) {
        dvv[i] = dd[k * NUP + lb * CB + i];
        su[i] = 0.f;
      }
#pragma unroll
      for (int j = 0; j < RB; ++j)
#pragma unroll
        for (int i = 0; i < CB; ++i) su[i] += Km[s2][i][j] * xv[j];
      red_a_all<CB>(su);
      if (la == 0)
#pragma unroll
        for (int i = 0; i < CB; ++i) utd[k * NUP + lb * CB + i] = dvv[i] + (double)su[i];
      wave_sync();
      if (k >= 1 && lane < NX) {
        const double xn = alpha * (double)xtf[k * NXP + lane] + oma * xd[k * NXP + lane];
        xd[k * NXP + lane] = xn;
        qtd[k * NXP + lane] = -qd[lane] * xrd[k * NXP + lane] - sigma * xn;
      }
      if (lane < M) {
        const int idx = k * M + lane;
        const double zeta = zc_s1 * utd[k * NUP + zc_i1] + zc_s2 * utd[k * NUP + zc_i2];
        const double wv = alpha * zeta + oma * zd[idx];
        const double zn = fmin(fmax(wv + yd[idx] * irhod[idx], lod[idx]), hid[idx]);
        const double yn = yd[idx] + rhod[idx] * (wv - zn);
        yd[idx] = yn;
        zd[idx] = zn;
        wvd[idx] = yn - rhod[idx] * zn;
      }
      if (lane < NU) {
        ud[k * NUP + lane] = alpha * utd[k * NUP + lane] + oma * ud[k * NUP + lane];
      }
      wave_sync();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    if (iters > 0) phaseA(I0{}, 1);
    if (iters > 0 && kS[0] == 0) {
      load_H(0);
      gprime0(1);
    }
    for (int it = 0; it < iters; ++it) {
      const int T = it + 1;
      if (hasH) {
        phaseA(I1{}, T);
        if (kS[1] == N - 1 && it >= 1) relax_xN(T - 1);
        load_H(kS[1]);
        flag_wait(sync + kStP + kS[1], 1, T, abortp, lane);
        phaseC(I1{}, T);
      }
      load_H(kS[0]);
      flag_wait(sync + kStP + kS[0], 1, T, abortp, lane);
      phaseC(I0{}, T);
      if (kS[0] >= 1) flag_wait(sync + kStX + kS[0], 1, T, abortp, lane);
      phaseE(I0{});
      if (it + 1 < iters) {
        phaseA(I0{}, T + 1);
        if (kS[0] == 0) gprime0(T + 1);  // H_0 is still in Hm from C_0
      }
      if (hasH) {
        flag_wait(sync + kStX + kS[1], 1, T, abortp, lane);
        phaseE(I1{});
      }
    }
    if (hasH && kS[1] == N - 1 && iters > 0) relax_xN(iters);
  }
  __syncthreads();

  bool fin = true;
  for (int i = tid; i < (N + 1) * NX; i += nt) {
    const float v = (float)xd[(i / NX) * NXP + i % NX];
    X[i] = v;
    fin &= (bool)isfinite(v);
  }
  for (int i = tid; i < N * NU; i += nt) {
    const float v = (float)ud[(i / NU) * NUP + i % NU];
    U[i] = v;
    fin &= (bool)isfinite(v);
  }
  for (int i = tid; i < N * M; i += nt) {
    Z[i] = (float)zd[i];
    Y[i] = (float)yd[i];
    fin &= (bool)isfinite(Z[i]) && (bool)isfinite(Y[i]);
  }
  if (!fin || sync[kStAbort]) atomicOr(flag, 1);
  __syncthreads();
  if (tid == 0 && flag[0]) st.status[agent] = AGENT_NONFINITE;
}

// One workgroup per agent of the launch list.
template <int NX, int NU, bool ROWS>
__global__ void __launch_bounds__(64 * kMaxStages)
k_admm_resident(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
                Inputs<float> in, SolverConsts sc_all, int iters, int warm,
                const float* __restrict__ fws, State<float> st) {
  if ((int)blockIdx.x >= n_launch) return;
  admm_resident_agent<NX, NU, ROWS>(desc, list ? list[blockIdx.x] : (int)blockIdx.x, in, sc_all, iters,
                                    warm, fws, st);
}

template <int NX, int NU>
__global__ void __launch_bounds__(64 * kMaxStages)
k_admm_stream(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
              Inputs<float> in, SolverConsts sc_all, int iters, int warm,
              const float* __restrict__ fws, State<float> st) {
  if ((int)blockIdx.x >= n_launch) return;
  admm_stream_agent<NX, NU>(desc, list ? list[blockIdx.x] : (int)blockIdx.x, in, sc_all, iters, warm,
                            fws, st);
}

// Persistent form: as many workgroups as the device holds at once, each
// taking the next agent of the list (longest horizon first) from a counter in
// device memory until the list is drained; an agent of horizon N <= 11 runs
// the register-resident body, a longer one the streaming body, in the same
// workgroup.  Every wavefront of the workgroup takes part in every agent
// (roles the agent does not need idle at its barriers), so the barriers
// between agents are met by all of them; the counter is zeroed by k_zero_counter
// on the same stream before the launch.
template <int NX, int NU>
__global__ void __launch_bounds__(64 * kMaxStages)
k_admm_persistent(const AgentDesc* __restrict__ desc, const int32_t* __restrict__ list, int n_launch,
                  Inputs<float> in, SolverConsts sc_all, int iters, int warm,
                  const float* __restrict__ fws, State<float> st, int* __restrict__ counter) {
  __shared__ int next;
  for (;;) {
    __syncthreads();  // the previous agent is written out before its LDS is reused
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = next;
    if (idx >= n_launch) break;
    __builtin_amdgcn_s_setprio(0);
    const int agent = list[idx];
    if (desc[agent].N + 1 <= kMaxStages)
      admm_resident_agent<NX, NU>(desc, agent, in, sc_all, iters, warm, fws, st);
    else
      admm_stream_agent<NX, NU>(desc, agent, in, sc_all, iters, warm, fws, st);
  }
}

__global__ void k_zero_counter(int* counter) { *counter = 0; }

// Workgroup size and dynamic LDS of a persistent launch whose longest horizon
// is N: enough wavefronts and LDS for the longest agent of either body.
template <int NX, int NU>
void persistent_shape(int N, int M, int* threads, size_t* lds) {
  const int nr = std::min(N, kMaxStages - 1);
  *threads = 64 * (nr + 1);
  *lds = iter_lds_layout<NX, NU>(nr, M).total;
  if (N + 1 > kMaxStages) {
    *threads = std::max(*threads, 64 * ((N + 1) / 2 + 2));
    *lds = std::max(*lds, (size_t)stream_lds_layout<NX, NU>(N, M).total);
  }
}

template <int NX, int NU>
hipError_t launch_pair(const AgentDesc* d_desc, const int32_t* list, int n_launch, int N, int M,
                       Inputs<float> in, SolverConsts sc, int iters, int warm, State<float> st,
                       float* fws, hipStream_t stream, int phase_mask, int* counter,
                       bool f32_products, int nc) {
  if (n_launch <= 0) return hipSuccess;
  const int lf = riccati_lds_bytes<NX, NU>();
  if (phase_mask & 1) {
    if (f32_products)
      hipLaunchKernelGGL((k_riccati<NX, NU, kProdF32, true>), dim3(n_launch), dim3(64 * kFactorWaves), lf,
                         stream, d_desc, list, n_launch, in, sc, fws, st.status);
    else
      hipLaunchKernelGGL((k_riccati<NX, NU, kProdF64, true>), dim3(n_launch), dim3(64 * kFactorWaves), lf,
                         stream, d_desc, list, n_launch, in, sc, fws, st.status);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((phase_mask & 2) && counter) {
    int threads = 0;
    size_t li = 0;
    persistent_shape<NX, NU>(N, M, &threads, &li);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(k_admm_persistent<NX, NU>), threads, li);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, std::min(n_launch, cus * std::max(per_cu, 1)));
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, stream, counter);
    hipLaunchKernelGGL((k_admm_persistent<NX, NU>), dim3(grid), dim3(threads), li, stream, d_desc, list,
                       n_launch, in, sc, iters, warm, fws, st, counter);
    return hipGetLastError();
  }
  if (phase_mask & 2) {
    if (N + 1 <= kMaxStages) {
      const int li = iter_lds_layout<NX, NU>(N, M, nc).total;
      if (nc)
        hipLaunchKernelGGL((k_admm_resident<NX, NU, true>), dim3(n_launch), dim3(64 * (N + 1)), li, stream,
                           d_desc, list, n_launch, in, sc, iters, warm, fws, st);
      else
        hipLaunchKernelGGL((k_admm_resident<NX, NU, false>), dim3(n_launch), dim3(64 * (N + 1)), li, stream,
                           d_desc, list, n_launch, in, sc, iters, warm, fws, st);
    } else {
      const int li = stream_lds_layout<NX, NU>(N, M).total;
      hipLaunchKernelGGL((k_admm_stream<NX, NU>), dim3(n_launch), dim3(64 * ((N + 1) / 2 + 2)), li, stream,
                         d_desc, list, n_launch, in, sc, iters, warm, fws, st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NX, int NU>
hipError_t set_limits() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdF64, true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdF32, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdF64, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdBF16, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdF16, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_riccati<NX, NU, kProdF32, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, riccati_lds_bytes<NX, NU>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_admm_resident<NX, NU, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_admm_resident<NX, NU, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_admm_stream<NX, NU>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  // the persistent kernel's own __shared__ word sits before the dynamic LDS
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_admm_persistent<NX, NU>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 16);
}

template <int NX, int NU>
int fused_lds(int N, int m, int nc = 0) {
  return N + 1 <= kMaxStages ? iter_lds_layout<NX, NU>(N, m, nc).total : stream_lds_layout<NX, NU>(N, m).total;
}

}  // namespace

bool fused_supported(int N, int nx, int nu, int n_feet, int nc) {
  const int m = nu + 4 * n_feet;
  if (N < 1 || N > kMaxStream || m > 64) return false;
  // the no-slip rows run on the register-resident body, and need a stage
  // before the last (the last stage's wavefront takes the rows of x_N)
  if (nc && (N < 2 || N + 1 > kMaxStages)) return false;
  if (nx == 48 && nu == 30) return fused_lds<48, 30>(N, m, nc) <= 160 * 1024;
  if (nx == 36 && nu == 24) return fused_lds<36, 24>(N, m, nc) <= 160 * 1024;
  return false;
}

void fused_launch_shape(int N, int nx, int nu, int n_feet, int* threads, size_t* lds, int nc) {
  const int m = nu + 4 * n_feet;
  *threads = N + 1 <= kMaxStages ? 64 * (N + 1) : 64 * ((N + 1) / 2 + 2);
  *lds = (nx == 48) ? fused_lds<48, 30>(N, m, nc) : fused_lds<36, 24>(N, m, nc);
  (void)nu;
}

size_t fused_agent_floats(int N, int nx, int nu) {
  (void)nu;
  // per stage: operator slots and s_k; per agent: S_0 (register-resident kernel)
  if (nx == 48) return (size_t)N * (FS<48, 30>::SLOTS * 64 + FS<48, 30>::NXP) + FS<48, 30>::AQ * 256;
  return (size_t)N * (FS<36, 24>::SLOTS * 64 + FS<36, 24>::NXP) + FS<36, 24>::AQ * 256;
}

hipError_t fused_set_limits() {
  hipError_t e = set_limits<48, 30>();
  if (e != hipSuccess) return e;
  return set_limits<36, 24>();
}

bool mixed_supported(int nx, int nu) { return (nx == 48 && nu == 30) || (nx == 36 && nu == 24); }

template <int X, int U, int P>
hipError_t launch_factor_generic_out(const AgentDesc* d_desc, const int32_t* list, int n_launch,
                                     Inputs<float> in, SolverConsts sc, float* ws,
                                     int32_t* status, hipStream_t stream) {
  const int lf = riccati_lds_bytes<X, U>();
  hipLaunchKernelGGL((k_riccati<X, U, P, false>), dim3(n_launch), dim3(64 * kFactorWaves), lf,
                     stream, d_desc, list, n_launch, in, sc, ws, status);
  return hipGetLastError();
}

hipError_t launch_mixed_factor(const AgentDesc* d_desc, const int32_t* list, int n_launch, int nx,
                               int nu, int prod, Inputs<float> in, SolverConsts sc, float* ws,
                               int32_t* status, hipStream_t stream) {
  if (n_launch <= 0) return hipSuccess;
  if (nx == 48 && nu == 30) {
    if (prod == kProdF64)
      return launch_factor_generic_out<48, 30, kProdF64>(d_desc, list, n_launch, in, sc, ws, status, stream);
    if (prod == kProdBF16)
      return launch_factor_generic_out<48, 30, kProdBF16>(d_desc, list, n_launch, in, sc, ws, status, stream);
    if (prod == kProdF32)
      return launch_factor_generic_out<48, 30, kProdF32>(d_desc, list, n_launch, in, sc, ws, status, stream);
    return launch_factor_generic_out<48, 30, kProdF16>(d_desc, list, n_launch, in, sc, ws, status, stream);
  }
  if (nx == 36 && nu == 24) {
    if (prod == kProdF64)
      return launch_factor_generic_out<36, 24, kProdF64>(d_desc, list, n_launch, in, sc, ws, status, stream);
    if (prod == kProdBF16)
      return launch_factor_generic_out<36, 24, kProdBF16>(d_desc, list, n_launch, in, sc, ws, status, stream);
    if (prod == kProdF32)
      return launch_factor_generic_out<36, 24, kProdF32>(d_desc, list, n_launch, in, sc, ws, status, stream);
    return launch_factor_generic_out<36, 24, kProdF16>(d_desc, list, n_launch, in, sc, ws, status, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t fused_solve_f32(const AgentDesc* d_desc, const int32_t* list, int n_launch, int N, int nx,
                           int nu, int n_feet, Inputs<float> in, SolverConsts sc, int iters,
                           int warm, State<float> st, float* fws, hipStream_t stream,
                           int phase_mask, int* counter, bool f32_products, int nc) {
  const int m = nu + 4 * n_feet;
  if (nc && (N + 1 > kMaxStages || counter)) return hipErrorInvalidValue;  // resident body only
  if (nx == 48 && nu == 30)
    return launch_pair<48, 30>(d_desc, list, n_launch, N, m, in, sc, iters, warm, st, fws, stream,
                               phase_mask, counter, f32_products, nc);
  if (nx == 36 && nu == 24)
    return launch_pair<36, 24>(d_desc, list, n_launch, N, m, in, sc, iters, warm, st, fws, stream,
                               phase_mask, counter, f32_products, nc);
  return hipErrorInvalidValue;
}

void fused_persistent_shape(int N, int nx, int nu, int n_feet, int* threads, size_t* lds) {
  const int m = nu + 4 * n_feet;
  if (nx == 48) persistent_shape<48, 30>(N, m, threads, lds);
  else persistent_shape<36, 24>(N, m, threads, lds);
}

}  // namespace mpc
