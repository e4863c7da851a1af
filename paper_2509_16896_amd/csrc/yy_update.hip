// yy_update.hip -- the online correction (Sec. 2.2 online stage, Sec. 9
// observation update) and the normalisation / estimation step (Sec. 2.2.2
// step 4, Sec. 9 normalisation), all in double precision with fixed-order
// reductions (no floating-point atomics), so repeated calls are bitwise equal.
#include <algorithm>
#include <cmath>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

// ---------------------------------------------------------------------------
// logw[i] += (h(x_i).dy - dt/2 |h(x_i)|^2) / rho2; one wavefront per node.
__global__ void __launch_bounds__(kBlock) k_loglik(int64_t n, int32_t r, int32_t m, int32_t obs,
                                                   const double* __restrict__ H, double h_shift,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ dy, double dt,
                                                   double rho2, double* __restrict__ logw) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const double li = logw[i];
    if (li == -INFINITY) continue;
    const double* xi = x + (size_t)i * r;
    double dot = 0.0, hh = 0.0;
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

// ---------------------------------------------------------------------------
// Normalisation.  Scratch layout (doubles): pmax[nb], psum[nb], pw2[nb],
// pmean[nb * r], sc[4] = {logZ, valid, 0, 0}.
__global__ void __launch_bounds__(kBlock) k_norm_max(int64_t n, const double* __restrict__ lw,
                                                     double* __restrict__ pmax) {
  __shared__ double sh[kBlock / 64];
  double m = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    m = fmax(m, lw[i]);
  m = block_max<kBlock>(m, sh);
  if (threadIdx.x == 0) pmax[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kBlock) k_norm_sumexp(int64_t n, int nb,
                                                        const double* __restrict__ pmax,
                                                        const double* __restrict__ lw,
                                                        double* __restrict__ psum) {
  __shared__ double sh[kBlock / 64];
  double M = -INFINITY;
  for (int p = threadIdx.x; p < nb; p += kBlock) M = fmax(M, pmax[p]);
  M = block_max<kBlock>(M, sh);
  double s = 0.0;
  if (M != -INFINITY)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
      s += exp(lw[i] - M);
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) psum[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_norm_logz(int nb, const double* __restrict__ pmax,
                                                      const double* __restrict__ psum,
                                                      double* __restrict__ sc,
                                                      double* __restrict__ logZ_step,
                                                      double* __restrict__ logZ_acc,
                                                      uint32_t* __restrict__ flags) {
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

// Block b handles rows [b*rows, (b+1)*rows): normalised log-weights, weights,
// partial sum of w^2 and partial weighted coordinate sums.
__global__ void __launch_bounds__(kBlock) k_norm_weights(int64_t n, int32_t r, int64_t rows,
                                                         const double* __restrict__ sc,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ lw,
                                                         double* __restrict__ w,
                                                         double* __restrict__ pw2,
                                                         double* __restrict__ pmean) {
  __shared__ double sw[kBlock];
  __shared__ double sh[kBlock / 64];
  if (sc[1] == 0.0) return;
  const double lz = sc[0];
  const int64_t b0 = (int64_t)blockIdx.x * rows;
  const int64_t b1 = std::min<int64_t>(b0 + rows, n);
  double w2 = 0.0;
  // per-thread accumulators for coordinates k = threadIdx.x + kBlock * c
  constexpr int kMaxC = 16;
  double acc[kMaxC];
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) acc[c] = 0.0;
  const int nc = (r + kBlock - 1) / kBlock;
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
    const int64_t cnt = std::min<int64_t>(kBlock, b1 - c0);
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
  w2 = block_sum<kBlock>(w2, sh);
  if (threadIdx.x == 0) pw2[blockIdx.x] = w2;
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) {
    const int k = threadIdx.x + kBlock * c;
    if (c < nc && k < r) pmean[(size_t)blockIdx.x * r + k] = acc[c];
  }
}

__global__ void __launch_bounds__(kBlock) k_norm_final(int nb, int32_t r, const double* __restrict__ sc,
                                                       const double* __restrict__ pw2,
                                                       const double* __restrict__ pmean,
                                                       double* __restrict__ mean,
                                                       double* __restrict__ ess) {
  if (sc[1] == 0.0) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < r) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += pmean[(size_t)b * r + k];
    mean[k] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += pw2[b];
    *ess = 1.0 / s;
  }
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
  int64_t blocks = (n + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  k_loglik<<<(unsigned)blocks, kBlock, 0, ctx->stream>>>(n, model->r, model->m, model->obs, model->H,
                                                         model->h_shift, x, dy, dt, model->rho2, logw);
  YY_LAUNCH_CHECK("k_loglik");
  return YY_OK;
}

extern "C" yy_status yy_normalise_moments(yy_ctx ctx, int64_t n, int32_t r, const double* x,
                                          double* logw, double* w, double* logZ_step,
                                          double* logZ_acc, double* mean, double* cov,
                                          double* ess) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_normalise_moments: ctx is NULL");
  if (n < 1) return fail(YY_ERR_ARG, "yy_normalise_moments: n < 1");
  if (r < 1 || r > 4096) return fail(YY_ERR_ARG, "yy_normalise_moments: r out of range");
  if (!x || !logw || !logZ_step || !logZ_acc || !mean || !ess)
    return fail(YY_ERR_ARG, "yy_normalise_moments: NULL array");
  YY_HIP(hipSetDevice(ctx->device));
  const int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 256);
  const int64_t rows = (n + nb - 1) / nb;
  const size_t need = (size_t)nb * (3 + (size_t)r) + 4 + (cov && !w ? (size_t)n : 0);
  yy_status st = ctx->red2.ensure(need * sizeof(double));
  if (st != YY_OK) return st;
  double* pmax = ctx->red2.as<double>();
  double* psum = pmax + nb;
  double* pw2 = psum + nb;
  double* pmean = pw2 + nb;
  double* sc = pmean + (size_t)nb * r;
  double* wbuf = w ? w : (cov ? sc + 4 : nullptr);
  k_norm_max<<<nb, kBlock, 0, ctx->stream>>>(n, logw, pmax);
  YY_LAUNCH_CHECK("k_norm_max");
  k_norm_sumexp<<<nb, kBlock, 0, ctx->stream>>>(n, nb, pmax, logw, psum);
  YY_LAUNCH_CHECK("k_norm_sumexp");
  k_norm_logz<<<1, kBlock, 0, ctx->stream>>>(nb, pmax, psum, sc, logZ_step, logZ_acc, ctx->d_flags);
  YY_LAUNCH_CHECK("k_norm_logz");
  k_norm_weights<<<nb, kBlock, 0, ctx->stream>>>(n, r, rows, sc, x, logw, wbuf, pw2, pmean);
  YY_LAUNCH_CHECK("k_norm_weights");
  k_norm_final<<<(r + kBlock - 1) / kBlock, kBlock, 0, ctx->stream>>>(nb, r, sc, pw2, pmean, mean, ess);
  YY_LAUNCH_CHECK("k_norm_final");
  if (cov) {
    dim3 grid((r + 63) / 64, (r + 63) / 64);
    k_norm_cov<<<grid, 256, 0, ctx->stream>>>(n, r, sc, x, wbuf, mean, cov);
    YY_LAUNCH_CHECK("k_norm_cov");
  }
  return YY_OK;
}
