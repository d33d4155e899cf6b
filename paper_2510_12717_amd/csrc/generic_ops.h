// Workgroup-level building blocks of the generic kernels (one workgroup per
// agent, up to 256 threads): finiteness checks, block reductions through LDS
// and quad-split dot products / matrix-vector products.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "xlane.h"

namespace mpc {

template <typename T>
__device__ inline bool finite_all(const T* p, int64_t n, int tid, int nt) {
  bool ok = true;
  for (int64_t i = tid; i < n; i += nt) ok &= (bool)isfinite(p[i]);
  return ok;
}

// Block-wide reductions through LDS (blockDim.x <= 256).
__device__ inline double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// A lane's terms are read in blocks of kQuadBlock: every load of a block is
// issued before the first is summed (indices past n_in are clamped to the last
// term, which is read and then not added, so no load sits behind a branch and
// waits alone).  The operators come from L2 or the infinity cache; summing each
// term as it arrived waited one memory latency per term (1.85x slower at the
// 4096-agent humanoid batch), and larger blocks cost occupancy.
constexpr int kQuadBlock = 8;

// init + the sum over t = t_first, t_first + step, ... < n of term(t), with
// kQuadBlock terms' loads in flight (indices past the end clamped, not added),
// added in increasing t: a single thread's (step 1) or a quad lane's (step 4)
// share of a dot product.
template <typename V, class FT>
__device__ inline V blocked_sum(int t_first, int step, int n, FT term, V init = V(0)) {
  V acc = init;
  for (int t0 = t_first; t0 < n; t0 += step * kQuadBlock) {
    V tv[kQuadBlock];
#pragma unroll
    for (int s = 0; s < kQuadBlock; ++s) tv[s] = term(min(t0 + step * s, n - 1));
#pragma unroll
    for (int s = 0; s < kQuadBlock; ++s) acc += t0 + step * s < n ? tv[s] : V(0);
  }
  return acc;
}

// store(i, sum_t term(i, t)) for i < n_out, t < n_in: each output's sum is
// split over the 4 lanes of a quad (terms t = sub, sub + 4, ...) and summed
// with DPP; each lane adds its terms in increasing t.
template <typename V, class FT, class FS>
__device__ inline void quad_dot(int n_out, int n_in, FT term, FS store, int tid, int nt) {
  const int qd = tid >> 2, sub = tid & 3, nq = nt >> 2;
  for (int i0 = 0; i0 < n_out; i0 += nq) {
    const int i = i0 + qd;
    if (i < n_out) {  // uniform within a quad
      V acc = 0;
      for (int t0 = sub; t0 < n_in; t0 += 4 * kQuadBlock) {
        V tv[kQuadBlock];
#pragma unroll
        for (int s = 0; s < kQuadBlock; ++s) tv[s] = term(i, min(t0 + 4 * s, n_in - 1));
#pragma unroll
        for (int s = 0; s < kQuadBlock; ++s) acc += t0 + 4 * s < n_in ? tv[s] : V(0);
      }
      acc = quad_sum(acc);
      if (sub == 0) store(i, acc);
    }
  }
}

// store(i, sum_t m(i, t) v_t) for i < n_out: each output's dot product is
// split over the 4 lanes of a quad (terms t = sub, sub + 4, ...) and summed
// with DPP, so a serial chain step costs n_in / 4 dependent FMAs.
template <typename V, class FM, class FS>
__device__ inline void quad_matvec(int n_out, int n_in, FM m, const V* v, FS store, int tid, int nt) {
  const int qd = tid >> 2, sub = tid & 3, nq = nt >> 2;
  for (int i0 = 0; i0 < n_out; i0 += nq) {
    const int i = i0 + qd;
    if (i < n_out) {  // uniform within a quad
      V acc = 0;
      for (int t0 = sub; t0 < n_in; t0 += 4 * kQuadBlock) {
        V mv[kQuadBlock], vv[kQuadBlock];
#pragma unroll
        for (int s = 0; s < kQuadBlock; ++s) {
          const int t = min(t0 + 4 * s, n_in - 1);
          mv[s] = (V)m(i, t);
          vv[s] = v[t];
        }
#pragma unroll
        for (int s = 0; s < kQuadBlock; ++s) acc += t0 + 4 * s < n_in ? mv[s] * vv[s] : V(0);
      }
      acc = quad_sum(acc);
      if (sub == 0) store(i, acc);
    }
  }
}

}  // namespace mpc
