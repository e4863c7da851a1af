// yy_update.hip -- the online correction (Sec. 2.2 online stage, Sec. 9
// observation update) and the normalisation / estimation step (Sec. 2.2.2
// step 4, Sec. 9 normalisation), all in double precision with fixed-order
// reductions (no floating-point atomics), so repeated calls are bitwise equal.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

// ---------------------------------------------------------------------------
// logw[i] += (h(x_i).dy - dt/2 |h(x_i)|^2) / rho2; one wavefront per node.
__device__ __forceinline__ void k_loglik_body(int64_t n, int32_t r, int32_t m, int32_t obs,
                                                   const double* __restrict__ H, double h_shift,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ dy, double dt,
                                                   double rho2, double* __restrict__ logw, int bx_, int gx_) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)bx_ * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gx_ * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const double li = logw[i];
    if (li == -INFINITY) continue;
    const double* xi = x + (size_t)i * r;
    double dot = 0.0, hh = 0.0;
    if (obs != YY_H_LINEAR && m == r && (r & 1) == 0 &&
        ((reinterpret_cast<uintptr_t>(xi) | reinterpret_cast<uintptr_t>(dy)) & 15) == 0) {
      // componentwise h on 16-byte pairs of coordinates
      const double2* x2 = reinterpret_cast<const double2*>(xi);
      const double2* d2 = reinterpret_cast<const double2*>(dy);
      for (int32_t k = lane; k < m / 2; k += 64) {
        const double2 v = x2[k], d = d2[k];
        double h0 = v.x, h1 = v.y;
        if (obs == YY_H_CUBE) {
          const double t0 = h0 - h_shift, t1 = h1 - h_shift;
          h0 = t0 * t0 * t0;
          h1 = t1 * t1 * t1;
        }
        dot = fma(h0, d.x, dot);
        hh = fma(h0, h0, hh);
        dot = fma(h1, d.y, dot);
        hh = fma(h1, h1, hh);
      }
      dot = wave_sum(dot);
      hh = wave_sum(hh);
      if (lane == 0) logw[i] = li + (dot - 0.5 * dt * hh) / rho2;
      continue;
    }
    for (int32_t k = lane; k < m; k += 64) {
      double h;
      if (obs == YY_H_IDENTITY) {
        h = xi[k];
      } else if (obs == YY_H_CUBE) {
        const double t = xi[k] - h_shift;
        h = t * t * t;
      } else {
        const double* Hk = H + (size_t)k * r;
        double acc = 0.0;
        for (int32_t l = 0; l < r; ++l) acc = fma(Hk[l], xi[l], acc);
        h = acc;
      }
      dot = fma(h, dy[k], dot);
      hh = fma(h, h, hh);
    }
    dot = wave_sum(dot);
    hh = wave_sum(hh);
    if (lane == 0) logw[i] = li + (dot - 0.5 * dt * hh) / rho2;
  }
}

__global__ void __launch_bounds__(kBlock) k_loglik(int64_t n, int32_t r, int32_t m, int32_t obs,
                                                   const double* __restrict__ H, double h_shift,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ dy, double dt,
                                                   double rho2, double* __restrict__ logw) {
  k_loglik_body(n, r, m, obs, H, h_shift, x, dy, dt, rho2, logw, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_loglik_batch(const loglik_args* __restrict__ A,
                                                         const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const loglik_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_loglik_body(a.n, a.r, a.m, a.obs, a.H, a.h_shift, a.x, a.kstep ? a.dy + (size_t)(*a.kstep - 1) * a.m : a.dy,
                a.dt, a.rho2, a.logw, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// ---------------------------------------------------------------------------
// Normalisation.  Scratch layout (doubles): pmax[nb], psum[nb], pw2[nb],
// pmean[nb * r], sc[4] = {logZ, valid, 0, 0}.
__device__ __forceinline__ void k_norm_max_body(int64_t n, const double* __restrict__ lw,
                                                     double* __restrict__ pmax, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  double m = -INFINITY;
  for (int64_t i = (int64_t)bx_ * kBlock + threadIdx.x; i < n; i += (int64_t)gx_ * kBlock)
    m = fmax(m, lw[i]);
  m = block_max<kBlock>(m, sh);
  if (threadIdx.x == 0) pmax[bx_] = m;
}

__global__ void __launch_bounds__(kBlock) k_norm_max(int64_t n, const double* __restrict__ lw,
                                                     double* __restrict__ pmax) {
  k_norm_max_body(n, lw, pmax, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_norm_max_batch(const norm_max_args* __restrict__ A,
                                                           const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const norm_max_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_norm_max_body(a.n, a.lw, a.pmax, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


__device__ __forceinline__ void k_norm_sumexp_body(int64_t n, int nb,
                                                        const double* __restrict__ pmax,
                                                        const double* __restrict__ lw,
                                                        double* __restrict__ psum, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  double M = -INFINITY;
  for (int p = threadIdx.x; p < nb; p += kBlock) M = fmax(M, pmax[p]);
  M = block_max<kBlock>(M, sh);
  double s = 0.0;
  if (M != -INFINITY)
    for (int64_t i = (int64_t)bx_ * kBlock + threadIdx.x; i < n; i += (int64_t)gx_ * kBlock)
      s += exp(lw[i] - M);
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) psum[bx_] = s;
}

__global__ void __launch_bounds__(kBlock) k_norm_sumexp(int64_t n, int nb,
                                                        const double* __restrict__ pmax,
                                                        const double* __restrict__ lw,
                                                        double* __restrict__ psum) {
  k_norm_sumexp_body(n, nb, pmax, lw, psum, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_norm_sumexp_batch(const norm_sumexp_args* __restrict__ A,
                                                              const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const norm_sumexp_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_norm_sumexp_body(a.n, a.nb, a.pmax, a.lw, a.psum, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


__device__ __forceinline__ void k_norm_logz_body(int nb, const double* __restrict__ pmax,
                                                      const double* __restrict__ psum,
                                                      double* __restrict__ sc,
                                                      double* __restrict__ logZ_step,
                                                      double* __restrict__ logZ_acc,
                                                      uint32_t* __restrict__ flags, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  double M = -INFINITY;
  for (int p = threadIdx.x; p < nb; p += kBlock) M = fmax(M, pmax[p]);
  M = block_max<kBlock>(M, sh);
  double s = 0.0;
  for (int p = threadIdx.x; p < nb; p += kBlock) s += psum[p];
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) {
    if (M == -INFINITY) {
      sc[0] = -INFINITY;
      sc[1] = 0.0;
      *logZ_step = -INFINITY;
      atomicOr(flags, YY_FLAG_ALL_ZERO);
    } else {
      const double lz = M + log(s);
      sc[0] = lz;
      sc[1] = 1.0;
      *logZ_step = lz;
      *logZ_acc += lz;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_norm_logz_batch(const norm_logz_args* __restrict__ A,
                                                            const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const norm_logz_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_norm_logz_body(a.nb, a.pmax, a.psum, a.sc, a.logZ_step, a.logZ_acc, a.flags, blockIdx.x - pre[q],
                   pre[q + 1] - pre[q]);
}


// Block b handles rows [b*rows, (b+1)*rows): normalised log-weights, weights,
// partial sum of w^2 and partial weighted coordinate sums, given logZ = lz.
__device__ __forceinline__ void k_norm_weights_core(int64_t n, int32_t r, int64_t rows, double lz,
                                                    const double* __restrict__ x, double* __restrict__ lw,
                                                    double* __restrict__ w, double* __restrict__ pw2,
                                                    double* __restrict__ pmean, int bx_, int gx_) {
  __shared__ double sw[kBlock];
  __shared__ double sh[kBlock / 64];
  const int64_t b0 = (int64_t)bx_ * rows;
  const int64_t b1 = std::min<int64_t>(b0 + rows, n);
  double w2 = 0.0;
  // per-thread accumulators for coordinates k = threadIdx.x + kBlock * c
  constexpr int kMaxC = 16;
  double acc[kMaxC];
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) acc[c] = 0.0;
  const int nc = (r + kBlock - 1) / kBlock;
  const bool pairs = (r & 1) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  // x NULL: no mean wanted, the pass over the coordinates is skipped
  const int64_t rows_x = x ? kBlock : 0;
  for (int64_t c0 = b0; c0 < b1; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    double wi = 0.0;
    if (i < b1) {
      const double l = lw[i] - lz;
      lw[i] = l;
      wi = exp(l);
      if (w) w[i] = wi;
      w2 = fma(wi, wi, w2);
    }
    __syncthreads();
    sw[threadIdx.x] = wi;
    __syncthreads();
    const int64_t cnt = std::min<int64_t>(rows_x, b1 - c0);
    if (pairs) {
      // 16-byte loads: thread j takes coordinates 2 (j + kBlock c) and 2 (j + kBlock c) + 1
      // (the same additions per coordinate in the same order as the scalar loop)
      for (int64_t t = 0; t < cnt; ++t) {
        const double wt = sw[t];
        const double2* xr = reinterpret_cast<const double2*>(x + (size_t)(c0 + t) * r);
#pragma unroll
        for (int c = 0; c < kMaxC / 2; ++c) {
          const int kk = threadIdx.x + kBlock * c;
          if (kk < r / 2) {
            const double2 v = xr[kk];
            acc[2 * c] = fma(wt, v.x, acc[2 * c]);
            acc[2 * c + 1] = fma(wt, v.y, acc[2 * c + 1]);
          }
        }
      }
    } else {
      for (int64_t t = 0; t < cnt; ++t) {
        const double wt = sw[t];
        const double* xr = x + (size_t)(c0 + t) * r;
#pragma unroll
        for (int c = 0; c < kMaxC; ++c) {
          const int k = threadIdx.x + kBlock * c;
          if (c < nc && k < r) acc[c] = fma(wt, xr[k], acc[c]);
        }
      }
    }
  }
  w2 = block_sum<kBlock>(w2, sh);
  if (threadIdx.x == 0) pw2[bx_] = w2;
  if (!x) return;
  if (pairs) {
#pragma unroll
    for (int c = 0; c < kMaxC / 2; ++c) {
      const int kk = threadIdx.x + kBlock * c;
      if (kk < r / 2) {
        pmean[(size_t)bx_ * r + 2 * kk] = acc[2 * c];
        pmean[(size_t)bx_ * r + 2 * kk + 1] = acc[2 * c + 1];
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < kMaxC; ++c) {
      const int k = threadIdx.x + kBlock * c;
      if (c < nc && k < r) pmean[(size_t)bx_ * r + k] = acc[c];
    }
  }
}

// The same with logZ read from sc (written by k_norm_logz; sc[1] = 0: nothing to do).
__device__ __forceinline__ void k_norm_weights_body(int64_t n, int32_t r, int64_t rows,
                                                    const double* __restrict__ sc, const double* __restrict__ x,
                                                    double* __restrict__ lw, double* __restrict__ w,
                                                    double* __restrict__ pw2, double* __restrict__ pmean, int bx_,
                                                    int gx_) {
  if (sc[1] == 0.0) return;
  k_norm_weights_core(n, r, rows, sc[0], x, lw, w, pw2, pmean, bx_, gx_);
}

// A single run's logZ and weights in one launch: every block forms logZ from the nb block
// maxima and sums with k_norm_logz_body's fixed-order reductions (the same value in every
// block; block 0 writes sc and the outputs, as k_norm_logz does), then its rows' weights.
__global__ void __launch_bounds__(kBlock) k_norm_logz_weights(int64_t n, int32_t r, int64_t rows, int nb,
                                                              const double* __restrict__ pmax,
                                                              const double* __restrict__ psum,
                                                              double* __restrict__ sc, double* __restrict__ logZ_step,
                                                              double* __restrict__ logZ_acc,
                                                              uint32_t* __restrict__ flags,
                                                              const double* __restrict__ x, double* __restrict__ lw,
                                                              double* __restrict__ w, double* __restrict__ pw2,
                                                              double* __restrict__ pmean) {
  __shared__ double sh[kBlock / 64];
  double M = -INFINITY;
  for (int p = threadIdx.x; p < nb; p += kBlock) M = fmax(M, pmax[p]);
  M = block_max<kBlock>(M, sh);
  double s = 0.0;
  for (int p = threadIdx.x; p < nb; p += kBlock) s += psum[p];
  s = block_sum<kBlock>(s, sh);
  const double lz = M == -INFINITY ? -INFINITY : M + log(s);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (M == -INFINITY) {
      sc[0] = -INFINITY;
      sc[1] = 0.0;
      *logZ_step = -INFINITY;
      atomicOr(flags, YY_FLAG_ALL_ZERO);
    } else {
      sc[0] = lz;
      sc[1] = 1.0;
      *logZ_step = lz;
      *logZ_acc += lz;
    }
  }
  if (M == -INFINITY) return;
  k_norm_weights_core(n, r, rows, lz, x, lw, w, pw2, pmean, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_norm_weights_batch(const norm_weights_args* __restrict__ A,
                                                               const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const norm_weights_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_norm_weights_body(a.n, a.r, a.rows, a.sc, a.x, a.lw, a.w, a.pw2, a.pmean, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// Sums of the per-block partials in a fixed order: block bx_ takes coordinates
// [kNormFinalK bx_, kNormFinalK (bx_ + 1)); its kNormFinalParts thread groups sum
// interleaved partial rows, and the group sums are added in group order.
constexpr int kNormFinalK = 32;
constexpr int kNormFinalParts = kBlock / kNormFinalK;
int norm_final_blocks(int32_t r) { return (r + kNormFinalK - 1) / kNormFinalK; }

__device__ __forceinline__ void k_norm_final_body(int nb, int32_t r, const double* __restrict__ sc,
                                                       const double* __restrict__ pw2,
                                                       const double* __restrict__ pmean,
                                                       double* __restrict__ mean,
                                                       double* __restrict__ ess, int bx_, int gx_) {
  __shared__ double sm[kNormFinalParts][kNormFinalK];
  __shared__ double se[kBlock];
  if (sc[1] == 0.0) return;
  const int kk = threadIdx.x % kNormFinalK, part = threadIdx.x / kNormFinalK;
  const int k = bx_ * kNormFinalK + kk;
  double s = 0.0;
  if (mean && k < r) {
    // (unrolled so that the loads of 8 partial rows are in flight at once; the
    // additions keep their order)
#pragma unroll 8
    for (int b = part; b < nb; b += kNormFinalParts) s += pmean[(size_t)b * r + k];
  }
  sm[part][kk] = s;
  if (bx_ == 0) {
    double e = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) e += pw2[b];
    se[threadIdx.x] = e;
  }
  __syncthreads();
  if (mean && part == 0 && k < r) {
    double t = 0.0;
    for (int p = 0; p < kNormFinalParts; ++p) t += sm[p][kk];
    mean[k] = t;
  }
  if (bx_ == 0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int p = 0; p < kBlock; ++p) t += se[p];
    *ess = 1.0 / t;
  }
}

__global__ void __launch_bounds__(kBlock) k_norm_final(int nb, int32_t r, const double* __restrict__ sc,
                                                       const double* __restrict__ pw2,
                                                       const double* __restrict__ pmean,
                                                       double* __restrict__ mean,
                                                       double* __restrict__ ess) {
  k_norm_final_body(nb, r, sc, pw2, pmean, mean, ess, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_norm_final_batch(const norm_final_args* __restrict__ A,
                                                             const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const norm_final_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_norm_final_body(a.nb, a.r, a.sc, a.pw2, a.pmean, a.mean, a.ess, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// Weighted covariance: 64 x 64 output tile per block (16 x 16 threads, 4 x 4
// each), all n rows in chunks of 16 staged through LDS.
__global__ void __launch_bounds__(256) k_norm_cov(int64_t n, int32_t r, const double* __restrict__ sc,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ mean,
                                                  double* __restrict__ cov) {
  __shared__ double sa[16][64];
  __shared__ double sb[16][64];
  __shared__ double sw[16];
  if (sc[1] == 0.0) return;
  const int a0 = blockIdx.y * 64, b0 = blockIdx.x * 64;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int64_t i0 = 0; i0 < n; i0 += 16) {
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int row = e >> 6, col = e & 63;
      const int64_t i = i0 + row;
      const int ka = a0 + col, kb = b0 + col;
      sa[row][col] = (i < n && ka < r) ? x[(size_t)i * r + ka] - mean[ka] : 0.0;
      sb[row][col] = (i < n && kb < r) ? x[(size_t)i * r + kb] - mean[kb] : 0.0;
    }
    if (threadIdx.x < 16) sw[threadIdx.x] = (i0 + threadIdx.x < n) ? w[i0 + threadIdx.x] : 0.0;
    __syncthreads();
#pragma unroll 4
    for (int t = 0; t < 16; ++t) {
      const double wt = sw[t];
      double va[4], vb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) va[p] = wt * sa[t][ty * 4 + p];
#pragma unroll
      for (int q = 0; q < 4; ++q) vb[q] = sb[t][tx * 4 + q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(va[p], vb[q], acc[p][q]);
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ka = a0 + ty * 4 + p, kb = b0 + tx * 4 + q;
      if (ka < r && kb < r) cov[(size_t)ka * r + kb] = acc[p][q];
    }
}


// Host launchers of the batched kernels (one block range per argument set).
yy_status launch_batched(hipStream_t st, const loglik_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_loglik_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_loglik_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const norm_max_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_norm_max_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_norm_max_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const norm_sumexp_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_norm_sumexp_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_norm_sumexp_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const norm_logz_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_norm_logz_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_norm_logz_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const norm_weights_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_norm_weights_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_norm_weights_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const norm_final_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_norm_final_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_norm_final_batch");
  return YY_OK;
}


// ---------------------------------------------------------------------------
// The correction and the normalisation in one pass over x (componentwise h,
// rows of even length): each wave takes rows of its block in turn, lane l
// holding the coordinate pairs l + 64 c (c < C) of the row in registers.  The
// row's log-likelihood term is summed in the order of k_loglik (the same
// updated log-weight), and its weight enters running sums relative to the
// wave's largest updated log-weight so far (rescaled when that grows).  Per
// block: its largest log-weight m_b, sum_i e^(l_i - m_b), sum_i e^(2(l_i - m_b))
// and sum_i e^(l_i - m_b) x_i, to part[b][3 + r].
template <int C>
__global__ void __launch_bounds__(kBlock) k_ln_partials(int64_t n, int32_t r, int64_t rows, int32_t obs,
                                                        double h_shift, const double* __restrict__ x,
                                                        const double* __restrict__ dy, double dt, double rho2,
                                                        double* __restrict__ logw, double* __restrict__ part) {
  constexpr int W = kBlock / 64;
  __shared__ double2 sdy[64 * C];
  __shared__ double red[W][2 * C * 64];
  __shared__ double sm[W][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int P = r >> 1;
  const double2* d2 = reinterpret_cast<const double2*>(dy);
  for (int p = threadIdx.x; p < 64 * C; p += kBlock) sdy[p] = p < P ? d2[p] : make_double2(0.0, 0.0);
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * rows;
  const int64_t b1 = b0 + rows < n ? b0 + rows : n;
  double acc[2 * C];
#pragma unroll
  for (int j = 0; j < 2 * C; ++j) acc[j] = 0.0;
  double m = -INFINITY, s = 0.0, s2 = 0.0;
  double2 v[C], vn[C];
  auto load = [&](int64_t i, double2(&o)[C]) {
    const double2* x2 = reinterpret_cast<const double2*>(x + (size_t)i * r);
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = lane + 64 * c < P ? x2[lane + 64 * c] : make_double2(0.0, 0.0);
  };
  int64_t i = b0 + wv;
  if (i < b1) load(i, v);
  for (; i < b1; i += W) {
    if (i + W < b1) load(i + W, vn);   // the wave's next row, in flight during this one
    const double li = logw[i];
    double dot = 0.0, hh = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double h0 = v[c].x, h1 = v[c].y;
      if (obs == YY_H_CUBE) {
        const double t0 = h0 - h_shift, t1 = h1 - h_shift;
        h0 = t0 * t0 * t0;
        h1 = t1 * t1 * t1;
      }
      if (lane + 64 * c >= P) {   // past the row: no term (h(0) need not vanish)
        h0 = 0.0;
        h1 = 0.0;
      }
      const double2 d = sdy[lane + 64 * c];
      dot = fma(h0, d.x, dot);
      hh = fma(h0, h0, hh);
      dot = fma(h1, d.y, dot);
      hh = fma(h1, h1, hh);
    }
    dot = wave_sum(dot);   // every lane holds the same sums
    hh = wave_sum(hh);
    if (li != -INFINITY) {
      const double l = li + (dot - 0.5 * dt * hh) / rho2;
      if (lane == 0) logw[i] = l;
      if (l > m) {
        const double f = exp(m - l);
        s *= f;
        s2 *= f * f;
#pragma unroll
        for (int j = 0; j < 2 * C; ++j) acc[j] *= f;
        m = l;
      }
      const double e = exp(l - m);
      s += e;
      s2 = fma(e, e, s2);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[2 * c] = fma(e, v[c].x, acc[2 * c]);
        acc[2 * c + 1] = fma(e, v[c].y, acc[2 * c + 1]);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = vn[c];
  }
  // the block's sums relative to its largest log-weight, waves added in order
  if (lane == 0) sm[wv][0] = m;
  __syncthreads();
  double mb = -INFINITY;
#pragma unroll
  for (int w = 0; w < W; ++w) mb = fmax(mb, sm[w][0]);
  const double f = m == -INFINITY ? 0.0 : exp(m - mb);
#pragma unroll
  for (int j = 0; j < 2 * C; ++j) red[wv][j * 64 + lane] = acc[j] * f;
  __syncthreads();
  if (lane == 0) {
    sm[wv][1] = s * f;
    sm[wv][2] = s2 * f * f;
  }
  __syncthreads();
  double* pb = part + (size_t)blockIdx.x * (3 + r);
  if (threadIdx.x == 0) {
    double a1 = 0.0, a2 = 0.0;
    for (int w = 0; w < W; ++w) {
      a1 += sm[w][1];
      a2 += sm[w][2];
    }
    pb[0] = mb;
    pb[1] = a1;
    pb[2] = a2;
  }
  for (int e = threadIdx.x; e < 2 * C * 64; e += kBlock) {
    const int j = e >> 6, l = e & 63;
    const int k = 2 * (l + 64 * (j >> 1)) + (j & 1);   // coordinate of accumulator j of lane l
    if (k < r) {
      double t = 0.0;
      for (int w = 0; w < W; ++w) t += red[w][e];
      pb[3 + k] = t;
    }
  }
}

// Every block first forms, from the nb block sums, M = max_b m_b, Z = sum_b e^(m_b - M) S_b
// and the factors e^(m_b - M) (fixed-order reductions, so every block gets the same values):
// logZ = M + log Z and the ESS Z^2 / sum_b e^(2(m_b - M)) S2_b, written by block 0 with
// sc = {logZ, valid, M, Z, then the factors}.  Then blocks [0, nfb): mean[k] =
// sum_b e^(m_b - M) part[b][3 + k] / Z in a fixed order (as k_norm_final); the others:
// logw -= logZ in place, w = e^logw.  (The scalars are formed in every block rather than in a
// one-block kernel before: that launch cost more than the repeated reduction over nb <= 1024.)
__global__ void __launch_bounds__(kBlock) k_ln_final(int64_t n, int nb, int32_t r, int nfb,
                                                     const double* __restrict__ part, double* __restrict__ sc,
                                                     double* __restrict__ logZ_step, double* __restrict__ logZ_acc,
                                                     double* __restrict__ ess, uint32_t* __restrict__ flags,
                                                     double* __restrict__ mean, double* __restrict__ logw,
                                                     double* __restrict__ w) {
  __shared__ double smn[kNormFinalParts][kNormFinalK];
  __shared__ double sh[kBlock / 64];
  __shared__ double sg[kMaxNormBlocks];
  const bool head = blockIdx.x == 0 && threadIdx.x == 0;
  const size_t stride = 3 + (size_t)r;
  double M = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += kBlock) M = fmax(M, part[b * stride]);
  M = block_max<kBlock>(M, sh);
  if (M == -INFINITY) {
    if (head) {
      sc[0] = -INFINITY;
      sc[1] = 0.0;
      *logZ_step = -INFINITY;
      atomicOr(flags, YY_FLAG_ALL_ZERO);
    }
    return;
  }
  double z = 0.0, z2 = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    const double g = exp(part[b * stride] - M);
    sg[b] = g;
    if (blockIdx.x == 0) sc[4 + b] = g;
    z = fma(g, part[b * stride + 1], z);
    z2 = fma(g * g, part[b * stride + 2], z2);
  }
  z = block_sum<kBlock>(z, sh);
  z2 = block_sum<kBlock>(z2, sh);   // (its barriers also publish sg)
  const double lz = M + log(z);
  if (head) {
    sc[0] = lz;
    sc[1] = 1.0;
    sc[2] = M;
    sc[3] = z;
    *logZ_step = lz;
    *logZ_acc += lz;
    *ess = z * z / z2;
  }
  if ((int)blockIdx.x >= nfb) {
    const int64_t nwb = (int64_t)gridDim.x - nfb;
    for (int64_t i = ((int64_t)blockIdx.x - nfb) * kBlock + threadIdx.x; i < n; i += nwb * kBlock) {
      const double l = logw[i] - lz;
      logw[i] = l;
      if (w) w[i] = exp(l);
    }
    return;
  }
  const int kk = threadIdx.x % kNormFinalK, pp = threadIdx.x / kNormFinalK;
  const int k = blockIdx.x * kNormFinalK + kk;
  double t = 0.0;
  if (k < r) {
    // (unrolled so that the loads of 8 partial rows are in flight at once; the additions keep their order)
#pragma unroll 8
    for (int b = pp; b < nb; b += kNormFinalParts) t = fma(sg[b], part[b * stride + 3 + k], t);
  }
  smn[pp][kk] = t;
  __syncthreads();
  if (pp == 0 && k < r) {
    double u = 0.0;
    for (int q = 0; q < kNormFinalParts; ++q) u += smn[q][kk];
    mean[k] = u / z;
  }
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_loglik_update(yy_ctx ctx, const yy_model* model, int64_t n, const double* x,
                                      const double* dy, double dt, double* logw) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_loglik_update: ctx is NULL");
  yy_status st = validate_model(model);
  if (st != YY_OK) return st;
  if (n < 0) return fail(YY_ERR_ARG, "yy_loglik_update: n < 0");
  if (!(dt > 0.0)) return fail(YY_ERR_ARG, "yy_loglik_update: dt must be positive");
  if (n == 0) return YY_OK;
  if (!x || !dy || !logw) return fail(YY_ERR_ARG, "yy_loglik_update: NULL array");
  YY_HIP(hipSetDevice(ctx->device));
  if (noise_b(model)) return noise_loglik(ctx, model, n, x, dy, dt, logw);   // b = V V^T (Sec. 7)
  int64_t blocks = (n + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  k_loglik<<<(unsigned)blocks, kBlock, 0, ctx->stream>>>(n, model->r, model->m, model->obs, model->H,
                                                         model->h_shift, x, dy, dt, model->rho2, logw);
  YY_LAUNCH_CHECK("k_loglik");
  return YY_OK;
}

namespace yy {

// The normalisation's launch sequence on a scratch area `red` of at least
// normalise_scratch_doubles(n, r, cov && !w) doubles (arguments checked by the caller).
static size_t normalise_scratch_doubles(int64_t n, int32_t r, bool own_w) {
  return (size_t)norm_blocks(n) * (3 + (size_t)r) + 4 + (own_w ? (size_t)n : 0);
}

static yy_status normalise_launch(yy_ctx ctx, int64_t n, int32_t r, const double* x, double* logw, double* w,
                                  double* logZ_step, double* logZ_acc, double* mean, double* cov, double* ess,
                                  double* red) {
  const int nb = norm_blocks(n);
  const int64_t rows = (n + nb - 1) / nb;
  double* pmax = red;
  double* psum = pmax + nb;
  double* pw2 = psum + nb;
  double* pmean = pw2 + nb;
  double* sc = pmean + (size_t)nb * r;
  double* wbuf = w ? w : (cov ? sc + 4 : nullptr);
  k_norm_max<<<nb, kBlock, 0, ctx->stream>>>(n, logw, pmax);
  YY_LAUNCH_CHECK("k_norm_max");
  k_norm_sumexp<<<nb, kBlock, 0, ctx->stream>>>(n, nb, pmax, logw, psum);
  YY_LAUNCH_CHECK("k_norm_sumexp");
  k_norm_logz_weights<<<nb, kBlock, 0, ctx->stream>>>(n, r, rows, nb, pmax, psum, sc, logZ_step, logZ_acc,
                                                       ctx->d_flags, mean ? x : nullptr, logw, wbuf, pw2, pmean);
  YY_LAUNCH_CHECK("k_norm_logz_weights");
  k_norm_final<<<mean ? norm_final_blocks(r) : 1, kBlock, 0, ctx->stream>>>(nb, r, sc, pw2, pmean, mean, ess);
  YY_LAUNCH_CHECK("k_norm_final");
  if (cov) {
    dim3 grid((r + 63) / 64, (r + 63) / 64);
    k_norm_cov<<<grid, 256, 0, ctx->stream>>>(n, r, sc, x, wbuf, mean, cov);
    YY_LAUNCH_CHECK("k_norm_cov");
  }
  return YY_OK;
}

static yy_status normalise_check(const char* who, yy_ctx ctx, int64_t n, int32_t r, const double* x,
                                 const double* logw, const double* logZ_step, const double* logZ_acc,
                                 const double* mean, const double* cov, const double* ess) {
  const std::string w(who);
  if (!ctx) return fail(YY_ERR_ARG, w + ": ctx is NULL");
  if (n < 1) return fail(YY_ERR_ARG, w + ": n < 1");
  if (r < 1 || r > 4096) return fail(YY_ERR_ARG, w + ": r out of range");
  if (!x || !logw || !logZ_step || !logZ_acc || !ess) return fail(YY_ERR_ARG, w + ": NULL array");
  if (!mean && cov) return fail(YY_ERR_ARG, w + ": cov needs mean");
  return YY_OK;
}

// ---------------------------------------------------------------------------
// Scratch of yy_normalise_moments_noalloc: the normalisation's per-block
// partial results (maximum, sum, sum of squared weights, weighted coordinate
// sums) and four scalars, for at most 1024 blocks and r <= YY_NOALLOC_MAX_R.
// One copy per GPU, held until the process ends.  Host code never passes
// `scratch` itself to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch_init).
constexpr size_t kNoallocDoubles = (size_t)1024 * (3 + YY_NOALLOC_MAX_R) + 4;
static __device__ __align__(256) double scratch[kNoallocDoubles];

constexpr int kNoallocDevices = 64;
static std::atomic<double*> g_scratch_ptr[kNoallocDevices];

yy_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoallocDevices) return YY_OK;   // the entry point reports it
  if (g_scratch_ptr[device].load(std::memory_order_acquire)) return YY_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device].store(static_cast<double*>(p), std::memory_order_release);
  return YY_OK;
}

}  // namespace yy

extern "C" yy_status yy_normalise_moments(yy_ctx ctx, int64_t n, int32_t r, const double* x,
                                          double* logw, double* w, double* logZ_step,
                                          double* logZ_acc, double* mean, double* cov,
                                          double* ess) {
  yy_status st = normalise_check("yy_normalise_moments", ctx, n, r, x, logw, logZ_step, logZ_acc, mean, cov, ess);
  if (st != YY_OK) return st;
  YY_HIP(hipSetDevice(ctx->device));
  if ((st = ctx->red2.ensure(normalise_scratch_doubles(n, r, cov && !w) * sizeof(double))) != YY_OK) return st;
  return normalise_launch(ctx, n, r, x, logw, w, logZ_step, logZ_acc, mean, cov, ess, ctx->red2.as<double>());
}

extern "C" yy_status yy_normalise_moments_noalloc(yy_ctx ctx, int64_t n, int32_t r, const double* x,
                                                  double* logw, double* w, double* logZ_step,
                                                  double* logZ_acc, double* mean, double* cov,
                                                  double* ess) {
  yy_status st =
      normalise_check("yy_normalise_moments_noalloc", ctx, n, r, x, logw, logZ_step, logZ_acc, mean, cov, ess);
  if (st != YY_OK) return st;
  if (r > YY_NOALLOC_MAX_R)
    return fail(YY_ERR_UNSUPPORTED, "yy_normalise_moments_noalloc: r = " + std::to_string(r) +
                                        " exceeds the static scratch's maximum " + std::to_string(YY_NOALLOC_MAX_R));
  if (cov && !w) return fail(YY_ERR_ARG, "yy_normalise_moments_noalloc: cov needs the caller's w");
  if (ctx->device < 0 || ctx->device >= kNoallocDevices)
    return fail(YY_ERR_UNSUPPORTED, "yy_normalise_moments_noalloc: device index beyond the scratch table");
  double* red = g_scratch_ptr[ctx->device].load(std::memory_order_acquire);
  if (!red) return fail(YY_ERR_HIP, "yy_normalise_moments_noalloc: static scratch not set up on this device");
  if (normalise_scratch_doubles(n, r, false) > kNoallocDoubles)
    return fail(YY_ERR_UNSUPPORTED, "yy_normalise_moments_noalloc: scratch too small");
  YY_HIP(hipSetDevice(ctx->device));
  return normalise_launch(ctx, n, r, x, logw, w, logZ_step, logZ_acc, mean, cov, ess, red);
}

extern "C" yy_status yy_loglik_normalise(yy_ctx ctx, const yy_model* model, int64_t n, const double* x,
                                         const double* dy, double dt, double* logw, double* w,
                                         double* logZ_step, double* logZ_acc, double* mean, double* ess) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_loglik_normalise: ctx is NULL");
  yy_status st = validate_model(model);
  if (st != YY_OK) return st;
  if (n < 1) return fail(YY_ERR_ARG, "yy_loglik_normalise: n < 1");
  if (!(dt > 0.0)) return fail(YY_ERR_ARG, "yy_loglik_normalise: dt must be positive");
  if (!x || !dy || !logw || !logZ_step || !logZ_acc || !mean || !ess)
    return fail(YY_ERR_ARG, "yy_loglik_normalise: NULL array");
  const int32_t r = model->r;
  const bool one_pass = model->obs != YY_H_LINEAR && model->m == r && (r & 1) == 0 && r <= 1024 && !noise_b(model) &&
                        ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(dy)) & 15) == 0;
  if (!one_pass) {
    if ((st = yy_loglik_update(ctx, model, n, x, dy, dt, logw)) != YY_OK) return st;
    return yy_normalise_moments(ctx, n, r, x, logw, w, logZ_step, logZ_acc, mean, nullptr, ess);
  }
  YY_HIP(hipSetDevice(ctx->device));
  const int nb = norm_blocks(n);
  const int64_t rows = (n + nb - 1) / nb;
  if ((st = ctx->red2.ensure(((size_t)nb * (4 + (size_t)r) + 4) * sizeof(double))) != YY_OK) return st;
  double* part = ctx->red2.as<double>();
  double* sc = part + (size_t)nb * (3 + r);
  const int P = r / 2;
  if (P <= 128) {
    k_ln_partials<2><<<nb, kBlock, 0, ctx->stream>>>(n, r, rows, model->obs, model->h_shift, x, dy, dt, model->rho2,
                                                     logw, part);
  } else if (P <= 256) {
    k_ln_partials<4><<<nb, kBlock, 0, ctx->stream>>>(n, r, rows, model->obs, model->h_shift, x, dy, dt, model->rho2,
                                                     logw, part);
  } else {
    k_ln_partials<8><<<nb, kBlock, 0, ctx->stream>>>(n, r, rows, model->obs, model->h_shift, x, dy, dt, model->rho2,
                                                     logw, part);
  }
  YY_LAUNCH_CHECK("k_ln_partials");
  const int nfb = norm_final_blocks(r);
  const int nwb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  k_ln_final<<<nfb + nwb, kBlock, 0, ctx->stream>>>(n, nb, r, nfb, part, sc, logZ_step, logZ_acc, ess,
                                                     ctx->d_flags, mean, logw, w);
  YY_LAUNCH_CHECK("k_ln_final");
  return YY_OK;
}
