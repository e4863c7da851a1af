// yy_common.h -- small device helpers shared by libyy's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace yy {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ inline int wave_or(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

// Argument set of block b in a batched launch: pre[0] = 0 < pre[1] < ... <
// pre[nr] are the running block counts of the sets; returns q with
// pre[q] <= b < pre[q + 1].
__device__ inline int batch_find(const int* __restrict__ pre, int nr, int b) {
  int lo = 0, hi = nr;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ inline uint16_t f32_to_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Merge two base-2 (running max, scaled sum) pairs.
__device__ inline void lse2_merge(float& M, float& S, float Mo, float So) {
  if (Mo == -INFINITY) return;
  if (M == -INFINITY) {
    M = Mo;
    S = So;
    return;
  }
  if (Mo > M) {
    S = S * exp2f(M - Mo) + So;
    M = Mo;
  } else {
    S = S + So * exp2f(Mo - M);
  }
}

// Block-wide fixed-order reductions for blocks of kBlock threads.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
    sh[0] = t;
  }
  __syncthreads();
  return sh[0];
}

template <int NT>
__device__ inline double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int i = 1; i < NT / 64; ++i) t = fmax(t, sh[i]);
    sh[0] = t;
  }
  __syncthreads();
  return sh[0];
}

}  // namespace yy
