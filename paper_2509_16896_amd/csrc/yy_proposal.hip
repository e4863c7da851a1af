// yy_proposal.hip -- the learned restart proposal: a small FP32 multilayer
// perceptron (r -> H -> H -> 2r, exact GELU) with hand-written forward,
// backward and Adam kernels, the sample moments that serve as its training
// targets, and the checks that decide between the learned and the plain
// restart box (the plain box is the restart of Sec. 6).
#include <cmath>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

constexpr double kKappa = 3.0;     // box half-width = kKappa standard deviations
constexpr double kV0Frac = 0.01;   // variance floor as a fraction of (R / kKappa)^2
constexpr double kB1 = 0.9, kB2 = 0.999, kAdamEps = 1e-8;

// ---------------------------------------------------------------------------
// Small GEMM: C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn], FP32 accumulation in increasing k.  64 x 64 tile
// per block of 256 threads (4 x 4 outputs each), K staged 16 at a time in LDS.
// Epilogues: 0 plain, 1 + bias[n], 2 + bias[n] then GELU (pre-activation to Z).
constexpr int kGT = 64, kGK = 16;

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk,
                                              int64_t sbn, const float* __restrict__ bias,
                                              float* __restrict__ C, int64_t ldc, float* __restrict__ Z) {
  __shared__ float As[kGK][kGT + 1];
  __shared__ float Bs[kGK][kGT + 1];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const int tm = (tid >> 4) * 4, tn = (tid & 15) * 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;          // 0 .. 1023
      const int am = e >> 4, ak = e & 15;   // A tile: 64 rows x 16 k
      const int gm = m0 + am, gk = k0 + ak;
      As[ak][am] = (gm < M && gk < K) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.f;
      const int bk = e >> 6, bn = e & 63;   // B tile: 16 k x 64 cols
      const int gk2 = k0 + bk, gn = n0 + bn;
      Bs[bk][bn] = (gk2 < K && gn < N) ? B[(int64_t)gk2 * sbk + (int64_t)gn * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gm = m0 + tm + i, gn = n0 + tn + j;
      if (gm >= M || gn >= N) continue;
      float v = acc[i][j];
      if (EPI >= 1) v += bias[gn];
      if (EPI == 2) {
        Z[(int64_t)gm * ldc + gn] = v;
        v = gelu_f(v);
      }
      C[(int64_t)gm * ldc + gn] = v;
    }
}

// One row (M = 1) with A and the columns of B contiguous in k: a wave per
// output, its lanes striding over k (the forward pass of one restart).
template <int EPI>
__global__ void __launch_bounds__(256) k_gemv(int N, int K, const float* __restrict__ A,
                                              const float* __restrict__ B, int64_t sbn,
                                              const float* __restrict__ bias, float* __restrict__ C,
                                              float* __restrict__ Z) {
  const int lane = threadIdx.x & 63;
  const int nn = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (nn >= N) return;
  const float* b = B + (int64_t)nn * sbn;
  float acc = 0.f;
  for (int k = lane; k < K; k += 64) acc = fmaf(A[k], b[k], acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    float v = acc;
    if (EPI >= 1) v += bias[nn];
    if (EPI == 2) {
      Z[nn] = v;
      v = gelu_f(v);
    }
    C[nn] = v;
  }
}

template <int EPI>
static yy_status gemm(hipStream_t st, int M, int N, int K, const float* A, int64_t sam, int64_t sak,
                      const float* B, int64_t sbk, int64_t sbn, const float* bias, float* C, int64_t ldc,
                      float* Z = nullptr) {
  if (M == 1 && sak == 1 && sbk == 1) {
    k_gemv<EPI><<<(unsigned)((N + 3) / 4), 256, 0, st>>>(N, K, A, B, sbn, bias, C, Z);
    YY_LAUNCH_CHECK("k_gemv");
    return YY_OK;
  }
  dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
  k_gemm<EPI><<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, bias, C, ldc, Z);
  YY_LAUNCH_CHECK("k_gemm");
  return YY_OK;
}

__global__ void __launch_bounds__(kBlock) k_to_f32(int64_t count, const double* __restrict__ in,
                                                   float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}

// dZ = dA * GELU'(Z), in place on dA.
__global__ void __launch_bounds__(kBlock) k_gelu_back(int64_t count, const float* __restrict__ Z,
                                                      float* __restrict__ dA) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) dA[i] *= gelu_grad_f(Z[i]);
}

// Column sums db[n] = sum_m dZ[m][n] (bias gradients), increasing m.
__global__ void __launch_bounds__(kBlock) k_colsum(int M, int N, const float* __restrict__ dZ,
                                                   float* __restrict__ db) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

// Loss terms and d loss / d outputs; per-block partial loss sums (FP64).
__global__ void __launch_bounds__(kBlock) k_loss(int B, int r, const float* __restrict__ out,
                                                 const double* __restrict__ xhat,
                                                 const double* __restrict__ mu,
                                                 const double* __restrict__ var, double R,
                                                 float* __restrict__ dout, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t total = (int64_t)B * r;
  double term = 0.0;
  if (e < total) {
    const int64_t b = e / r, d = e % r;
    const double delta = out[b * 2 * r + d], u = out[b * 2 * r + r + d];
    const double s0 = R / kKappa;
    const double s = s0 * exp(u), s2 = s * s;
    const double err = mu[e] - xhat[e] - delta;
    const double A = var[e] + kV0Frac * s0 * s0 + err * err;
    term = A / (2.0 * s2) + log(s0) + u;
    const double inv = 1.0 / (double)total;
    dout[b * 2 * r + d] = (float)(-err / s2 * inv);
    dout[b * 2 * r + r + d] = (float)((1.0 - A / s2) * inv);
  }
  const double t = block_sum<kBlock>(term, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_loss_final(int nb, int64_t total, const double* __restrict__ part, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *loss = s / (double)total;
}

__global__ void __launch_bounds__(kBlock) k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, float lr,
                                                 float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = (float)kB1 * m[i] + (float)(1.0 - kB1) * gi;
  const float vi = (float)kB2 * v[i] + (float)(1.0 - kB2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + (float)kAdamEps);
}

// Default initialisation: uniform in +-bound from SplitMix64(seed, index).
__global__ void __launch_bounds__(kBlock) k_init_uniform(int64_t count, float* __restrict__ w, float bound,
                                                         uint64_t seed, uint64_t offset) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  uint64_t z = seed + ((uint64_t)(offset + i) + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * 0x1p-53;   // [0, 1)
  w[i] = (float)((2.0 * u - 1.0) * bound);
}

static unsigned nblk(int64_t count) { return (unsigned)((count + kBlock - 1) / kBlock); }

// Work buffers for B rows: x32 [B r], Z1, A1, Z2, A2 [B H], O, dO [B 2r], dA2/dZ2, dA1/dZ1 [B H].
struct Work {
  float *x32, *Z1, *A1, *Z2, *A2, *O, *dO, *d2, *d1;
};

static yy_status work_for(yy_proposal p, int32_t B, Work& w) {
  const int64_t r = p->r, H = p->H;
  const int64_t per = r + 4 * H + 4 * r + 2 * H;
  yy_status st = p->work.ensure((size_t)B * per * sizeof(float));
  if (st != YY_OK) return st;
  float* b = p->work.as<float>();
  w.x32 = b;
  w.Z1 = w.x32 + (size_t)B * r;
  w.A1 = w.Z1 + (size_t)B * H;
  w.Z2 = w.A1 + (size_t)B * H;
  w.A2 = w.Z2 + (size_t)B * H;
  w.O = w.A2 + (size_t)B * H;
  w.dO = w.O + (size_t)B * 2 * r;
  w.d2 = w.dO + (size_t)B * 2 * r;
  w.d1 = w.d2 + (size_t)B * H;
  return YY_OK;
}

static yy_status forward(yy_proposal p, int32_t B, const double* xhat, const Work& w) {
  hipStream_t st = p->ctx->stream;
  const int r = p->r, H = p->H;
  const float* P = p->pf();
  k_to_f32<<<nblk((int64_t)B * r), kBlock, 0, st>>>((int64_t)B * r, xhat, w.x32);
  YY_LAUNCH_CHECK("k_to_f32");
  yy_status s;
  // Z1 = x W1^T + b1, A1 = GELU(Z1)
  if ((s = gemm<2>(st, B, H, r, w.x32, r, 1, P + p->oW1, 1, r, P + p->ob1, w.A1, H, w.Z1)) != YY_OK) return s;
  if ((s = gemm<2>(st, B, H, H, w.A1, H, 1, P + p->oW2, 1, H, P + p->ob2, w.A2, H, w.Z2)) != YY_OK) return s;
  return gemm<1>(st, B, 2 * r, H, w.A2, H, 1, P + p->oW3, 1, H, P + p->ob3, w.O, 2 * r);
}

// Gradient of the loss w.r.t. the parameters into g, given dO in the work buffers.
static yy_status backward(yy_proposal p, int32_t B, const Work& w, float* g) {
  hipStream_t st = p->ctx->stream;
  const int r = p->r, H = p->H;
  const float* P = p->pf();
  yy_status s;
  // gW3[n][k] = sum_m dO[m][n] A2[m][k]; gb3 = colsum dO
  if ((s = gemm<0>(st, 2 * r, H, B, w.dO, 1, 2 * r, w.A2, H, 1, nullptr, g + p->oW3, H)) != YY_OK) return s;
  k_colsum<<<nblk(2 * r), kBlock, 0, st>>>(B, 2 * r, w.dO, g + p->ob3);
  YY_LAUNCH_CHECK("k_colsum");
  // dA2 = dO W3; dZ2 = dA2 GELU'(Z2)
  if ((s = gemm<0>(st, B, H, 2 * r, w.dO, 2 * r, 1, P + p->oW3, H, 1, nullptr, w.d2, H)) != YY_OK) return s;
  k_gelu_back<<<nblk((int64_t)B * H), kBlock, 0, st>>>((int64_t)B * H, w.Z2, w.d2);
  YY_LAUNCH_CHECK("k_gelu_back");
  if ((s = gemm<0>(st, H, H, B, w.d2, 1, H, w.A1, H, 1, nullptr, g + p->oW2, H)) != YY_OK) return s;
  k_colsum<<<nblk(H), kBlock, 0, st>>>(B, H, w.d2, g + p->ob2);
  YY_LAUNCH_CHECK("k_colsum");
  // dA1 = dZ2 W2; dZ1 = dA1 GELU'(Z1)
  if ((s = gemm<0>(st, B, H, H, w.d2, H, 1, P + p->oW2, H, 1, nullptr, w.d1, H)) != YY_OK) return s;
  k_gelu_back<<<nblk((int64_t)B * H), kBlock, 0, st>>>((int64_t)B * H, w.Z1, w.d1);
  YY_LAUNCH_CHECK("k_gelu_back");
  if ((s = gemm<0>(st, H, r, B, w.d1, 1, H, w.x32, r, 1, nullptr, g + p->oW1, r)) != YY_OK) return s;
  k_colsum<<<nblk(H), kBlock, 0, st>>>(B, H, w.d1, g + p->ob1);
  YY_LAUNCH_CHECK("k_colsum");
  return YY_OK;
}

// ---------------------------------------------------------------------------
// Restart checks.  dec[0] = learned box passed coverage and log-density,
// dec[1] = the plain nodes must be regenerated (the ESS check failed),
// dec[2] = the learned box was used.  box (device [5r] doubles): learned
// lo, hi, then the centre, the half-width and kappa / half-width (the inverse
// standard deviation) of the learned box.

// One wavefront per distinct resampled node (a run of equal ancestors), its
// terms counted with the run's length: counts of coordinates inside the
// learned box and the sums of squared standardised deviations under both boxes
// (the log terms of the densities do not depend on the sample and are added
// once in k_prop_decide); per-block partials.
__global__ void __launch_bounds__(kBlock) k_prop_checks(int64_t n, int32_t r, const double* __restrict__ x,
                                                        const int64_t* __restrict__ idx,
                                                        const double* __restrict__ mean, double R,
                                                        const double* __restrict__ box,
                                                        double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  const int lane = threadIdx.x & 63;
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t wave = gt >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const double* c = box + 2 * r;
  const double* hw = box + 3 * r;
  const double* isL = box + 4 * r;
  const double isP = kKappa / R;
  double cov = 0.0, qL = 0.0, qP = 0.0;
  double c1 = 0.0, l1 = 0.0, p1 = 0.0;   // one sample's terms
  auto coord = [&](double yd, double cd, double hd, double id, double md) {
    const double zl = (yd - cd) * id, zp = (yd - md) * isP;
    c1 += fabs(yd - cd) <= hd ? 1.0 : 0.0;
    l1 = fma(zl, zl, l1);
    p1 = fma(zp, zp, p1);
  };
  // 16-byte accesses to pairs of coordinates when the rows allow it
  const bool pairs = (r & 1) == 0 && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(box) |
                                       reinterpret_cast<uintptr_t>(mean)) & 15) == 0;
  // the box and the mean staged in LDS for rows of up to 2 kStagePairs coordinates (every
  // resampled row reads them all)
  constexpr int kStagePairs = 512;
  __shared__ double2 s_c[kStagePairs], s_h[kStagePairs], s_i[kStagePairs], s_m[kStagePairs];
  const bool staged = pairs && r <= 2 * kStagePairs;
  if (staged) {
    for (int p = threadIdx.x; p < r / 2; p += kBlock) {
      s_c[p] = reinterpret_cast<const double2*>(c)[p];
      s_h[p] = reinterpret_cast<const double2*>(hw)[p];
      s_i[p] = reinterpret_cast<const double2*>(isL)[p];
      s_m[p] = reinterpret_cast<const double2*>(mean)[p];
    }
    __syncthreads();
  }
  // The systematic resampling's ancestors are non-decreasing, so equal ones are contiguous: each
  // distinct ancestor is read once and its terms count with their multiplicity (the first sample of
  // a run finds the run's end by bisection).
  for (int64_t t = wave; t < n; t += nwaves) {
    const int64_t it = idx[t];
    if (t > 0 && idx[t - 1] == it) continue;
    int64_t lo = t + 1, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (idx[mid] == it) lo = mid + 1;
      else hi = mid;
    }
    const double mult = (double)(lo - t);
    const double* y = x + (size_t)it * r;
    c1 = 0.0;
    l1 = 0.0;
    p1 = 0.0;
    if (staged) {
      const double2* y2 = reinterpret_cast<const double2*>(y);
      for (int32_t d = lane; d < r / 2; d += 64) {
        const double2 yd = y2[d], cd = s_c[d], hd = s_h[d], id = s_i[d], md = s_m[d];
        coord(yd.x, cd.x, hd.x, id.x, md.x);
        coord(yd.y, cd.y, hd.y, id.y, md.y);
      }
    } else if (pairs) {
      const double2* y2 = reinterpret_cast<const double2*>(y);
      for (int32_t d = lane; d < r / 2; d += 64) {
        const double2 yd = y2[d], cd = reinterpret_cast<const double2*>(c)[d];
        const double2 hd = reinterpret_cast<const double2*>(hw)[d], id = reinterpret_cast<const double2*>(isL)[d];
        const double2 md = reinterpret_cast<const double2*>(mean)[d];
        coord(yd.x, cd.x, hd.x, id.x, md.x);
        coord(yd.y, cd.y, hd.y, id.y, md.y);
      }
    } else {
      for (int32_t d = lane; d < r; d += 64) coord(y[d], c[d], hw[d], isL[d], mean[d]);
    }
    cov = fma(mult, c1, cov);
    qL = fma(mult, l1, qL);
    qP = fma(mult, p1, qP);
  }
  const double ldL = qL, ldP = qP;
  const double a = block_sum<kBlock>(cov, sh);
  const double b = block_sum<kBlock>(ldL, sh);
  const double e = block_sum<kBlock>(ldP, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = e;
  }
}

// Learned box from the network outputs (FP64 from the FP32 outputs).
__global__ void __launch_bounds__(kBlock) k_prop_box(int32_t r, const float* __restrict__ out,
                                                     const double* __restrict__ mean, double R,
                                                     double* __restrict__ box) {
  const int d = blockIdx.x * kBlock + threadIdx.x;
  if (d >= r) return;
  const double c = mean[d] + (double)out[d];
  const double hw = R * exp((double)out[r + d]);
  box[d] = c - hw;
  box[r + d] = c + hw;
  box[2 * r + d] = c;
  box[3 * r + d] = hw;
  box[4 * r + d] = kKappa / hw;
}

// Decision on coverage and log-density; writes the chosen box.
__global__ void __launch_bounds__(kBlock) k_prop_decide(int nb, int64_t n, int32_t r, double cover_min,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ mean, double R,
                                                        const double* __restrict__ box,
                                                        double* __restrict__ box_lo, double* __restrict__ box_hi,
                                                        int* __restrict__ dec) {
  __shared__ int ok;
  __shared__ double sa[kBlock], sq[kBlock], sp[kBlock], sl[kBlock];
  // partial sums in a fixed order: thread k takes partials k, k + kBlock, ...
  // (and coordinates k, k + kBlock, ... of the log standard deviations), then
  // thread 0 adds the thread sums in thread order
  double a = 0.0, qL = 0.0, qP = 0.0, lg = 0.0;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a += part[3 * k];
    qL += part[3 * k + 1];
    qP += part[3 * k + 2];
  }
  for (int d = threadIdx.x; d < r; d += kBlock) lg += log(box[3 * r + d] / kKappa);
  sa[threadIdx.x] = a;
  sq[threadIdx.x] = qL;
  sp[threadIdx.x] = qP;
  sl[threadIdx.x] = lg;
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, QL = 0.0, QP = 0.0, LG = 0.0;
    for (int k = 0; k < kBlock; ++k) {
      A += sa[k];
      QL += sq[k];
      QP += sp[k];
      LG += sl[k];
    }
    // mean log-densities of the samples under the two diagonal Gaussians,
    // constant terms common to both dropped
    const double b = -0.5 * QL - (double)n * LG;
    const double e = -0.5 * QP - (double)n * (double)r * log(R / kKappa);
    ok = (A / ((double)n * (double)r) >= cover_min) && (b >= e);
    dec[0] = ok;
    dec[1] = 0;
    dec[2] = 0;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < r; d += kBlock) {
    box_lo[d] = ok ? box[d] : __dsub_rn(mean[d], R);
    box_hi[d] = ok ? box[r + d] : __dadd_rn(mean[d], R);
  }
}

// Prior ESS of the new nodes: per-block max, then per-block sums of e^{l-M}, e^{2(l-M)}.
__global__ void __launch_bounds__(kBlock) k_prior_max(int64_t n, const double* __restrict__ lw,
                                                      double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double m = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    m = fmax(m, lw[i]);
  m = block_max<kBlock>(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kBlock) k_prior_sums(int64_t n, int nb, const double* __restrict__ lw,
                                                       double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double M = -INFINITY;
  for (int k = 0; k < nb; ++k) M = fmax(M, part[k]);
  double s1 = 0.0, s2 = 0.0;
  if (M != -INFINITY) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
      const double l = lw[i];
      if (l == -INFINITY) continue;
      const double e = exp(l - M);
      s1 += e;
      s2 += e * e;
    }
  }
  const double a = block_sum<kBlock>(s1, sh);
  const double b = block_sum<kBlock>(s2, sh);
  if (threadIdx.x == 0) {
    part[nb + 2 * blockIdx.x] = a;
    part[nb + 2 * blockIdx.x + 1] = b;
  }
}

__global__ void __launch_bounds__(kBlock) k_prop_final(int nb, int32_t r, double ess_min,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ mean, double R,
                                                       double* __restrict__ box_lo, double* __restrict__ box_hi,
                                                       int* __restrict__ dec, int32_t* __restrict__ used,
                                                       uint32_t* __restrict__ flags) {
  __shared__ int redo;
  if (threadIdx.x == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nb; ++k) {
      s1 += part[nb + 2 * k];
      s2 += part[nb + 2 * k + 1];
    }
    const double ess = s2 > 0.0 ? s1 * s1 / s2 : 0.0;
    const int ok = dec[0] && ess >= ess_min;
    redo = dec[0] && !ok;
    dec[1] = redo;
    dec[2] = ok;
    if (used) *used = ok;
    if (!ok) atomicOr(flags, YY_FLAG_PROPOSAL_FALLBACK);
  }
  __syncthreads();
  if (redo)
    for (int d = threadIdx.x; d < r; d += kBlock) {
      box_lo[d] = __dsub_rn(mean[d], R);
      box_hi[d] = __dadd_rn(mean[d], R);
    }
}

// Sample moments of x[idx[t]]: per-coordinate sums in fixed order.  One thread
// per coordinate d walks t = 0 .. n-1 in chunks: partial sums per chunk go to
// part[chunk][r], summed afterwards in chunk order.
constexpr int64_t kMomChunk = 1024;

__global__ void __launch_bounds__(kBlock) k_mom_pass(int64_t n, int32_t r, const double* __restrict__ x,
                                                     const int64_t* __restrict__ idx,
                                                     const double* __restrict__ mean, double* __restrict__ part) {
  const int d = blockIdx.x * kBlock + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (d >= r) return;
  const int64_t t0 = chunk * kMomChunk, t1 = t0 + kMomChunk < n ? t0 + kMomChunk : n;
  double s = 0.0;
  if (!mean) {
    for (int64_t t = t0; t < t1; ++t) s += x[(size_t)idx[t] * r + d];
  } else {
    const double m = mean[d];
    for (int64_t t = t0; t < t1; ++t) {
      const double e = x[(size_t)idx[t] * r + d] - m;
      s += e * e;
    }
  }
  part[(size_t)chunk * r + d] = s;
}

__global__ void __launch_bounds__(kBlock) k_mom_reduce(int64_t n, int32_t r, int64_t nchunk,
                                                       const double* __restrict__ part, double* __restrict__ out) {
  const int d = blockIdx.x * kBlock + threadIdx.x;
  if (d >= r) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += part[(size_t)c * r + d];
  out[d] = s / (double)n;
}

yy_status proposal_restart_prepare(yy_ctx ctx, yy_proposal p, int64_t n, int32_t r, const double* x_cur,
                                   const int64_t* idx, const double* mean, double R, double cover_min,
                                   double* box_lo, double* box_hi, int** dec_out) {
  hipStream_t st = ctx->stream;
  Work w;
  yy_status s = work_for(p, 1, w);
  if (s != YY_OK) return s;
  int nb = (int)((n * 64 + kBlock - 1) / kBlock);
  if (nb > 2048) nb = 2048;
  // part: box [5r] + check partials [3 nb] + ESS partials [3 nb] + decision ints
  const size_t need = (5 * (size_t)r + 6 * (size_t)nb + 4) * sizeof(double);
  if ((s = p->part.ensure(need)) != YY_OK) return s;
  double* box = p->part.as<double>();
  double* cpart = box + 5 * (size_t)r;
  int* dec = reinterpret_cast<int*>(cpart + 6 * (size_t)nb);
  if ((s = forward(p, 1, mean, w)) != YY_OK) return s;
  k_prop_box<<<nblk(r), kBlock, 0, st>>>(r, w.O, mean, R, box);
  YY_LAUNCH_CHECK("k_prop_box");
  k_prop_checks<<<nb, kBlock, 0, st>>>(n, r, x_cur, idx, mean, R, box, cpart);
  YY_LAUNCH_CHECK("k_prop_checks");
  k_prop_decide<<<1, kBlock, 0, st>>>(nb, n, r, cover_min, cpart, mean, R, box, box_lo, box_hi, dec);
  YY_LAUNCH_CHECK("k_prop_decide");
  *dec_out = dec;
  return YY_OK;
}

yy_status proposal_restart_finish(yy_ctx ctx, yy_proposal p, int64_t n, int32_t r, const double* lw_new,
                                  const double* mean, double R, double ess_min, double* box_lo,
                                  double* box_hi, int* dec, int32_t* used) {
  hipStream_t st = ctx->stream;
  int nb = (int)((n + kBlock - 1) / kBlock);
  if (nb > 1024) nb = 1024;
  double* part = p->part.as<double>() + 5 * (size_t)r;   // reuses the check partials (3 nb >= nb + 2 nb)
  k_prior_max<<<nb, kBlock, 0, st>>>(n, lw_new, part);
  YY_LAUNCH_CHECK("k_prior_max");
  k_prior_sums<<<nb, kBlock, 0, st>>>(n, nb, lw_new, part);
  YY_LAUNCH_CHECK("k_prior_sums");
  k_prop_final<<<1, kBlock, 0, st>>>(nb, r, ess_min, part, mean, R, box_lo, box_hi, dec, used, ctx->d_flags);
  YY_LAUNCH_CHECK("k_prop_final");
  return YY_OK;
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_proposal_create(yy_ctx ctx, int32_t r, int32_t hidden, uint64_t seed,
                                        const float* params, yy_proposal* out) {
  if (!ctx || !out) return fail(YY_ERR_ARG, "yy_proposal_create: NULL argument");
  if (r < 1 || r > YY_MAX_R) return fail(YY_ERR_ARG, "yy_proposal_create: r out of range");
  if (hidden < 1 || hidden > 1024) return fail(YY_ERR_ARG, "yy_proposal_create: hidden out of range");
  YY_HIP(hipSetDevice(ctx->device));
  yy_proposal p = new yy_proposal_s();
  p->ctx = ctx;
  p->r = r;
  p->H = hidden;
  const int64_t H = hidden;
  p->oW1 = 0;
  p->ob1 = p->oW1 + H * r;
  p->oW2 = p->ob1 + H;
  p->ob2 = p->oW2 + H * H;
  p->oW3 = p->ob2 + H;
  p->ob3 = p->oW3 + 2 * (int64_t)r * H;
  p->P = p->ob3 + 2 * (int64_t)r;
  const size_t bytes = (size_t)p->P * sizeof(float);
  yy_status s;
  if ((s = p->params.ensure(bytes)) != YY_OK || (s = p->adam_m.ensure(bytes)) != YY_OK ||
      (s = p->adam_v.ensure(bytes)) != YY_OK || (s = p->grad.ensure(bytes)) != YY_OK) {
    delete p;
    return s;
  }
  hipStream_t st = ctx->stream;
  if (params) {
    if (hipMemcpyAsync(p->pf(), params, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      delete p;
      return fail(YY_ERR_HIP, "yy_proposal_create: copy of params failed");
    }
  } else {
    if (hipMemsetAsync(p->pf(), 0, bytes, st) != hipSuccess) {
      delete p;
      return fail(YY_ERR_HIP, "yy_proposal_create: memset failed");
    }
    k_init_uniform<<<nblk(H * r), kBlock, 0, st>>>(H * r, p->pf() + p->oW1, (float)(1.0 / std::sqrt((double)r)),
                                                   seed, 0);
    k_init_uniform<<<nblk(H * H), kBlock, 0, st>>>(H * H, p->pf() + p->oW2, (float)(1.0 / std::sqrt((double)H)),
                                                   seed, (uint64_t)(H * r));
  }
  if (hipMemsetAsync(p->adam_m.ptr, 0, bytes, st) != hipSuccess ||
      hipMemsetAsync(p->adam_v.ptr, 0, bytes, st) != hipSuccess) {
    delete p;
    return fail(YY_ERR_HIP, "yy_proposal_create: memset failed");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "yy_proposal_create");
  }
  *out = p;
  return YY_OK;
}

extern "C" yy_status yy_proposal_destroy(yy_proposal p) {
  if (!p) return YY_OK;
  if (p->ctx) {
    hipSetDevice(p->ctx->device);
    hipStreamSynchronize(p->ctx->stream);
  }
  p->params.release();
  p->adam_m.release();
  p->adam_v.release();
  p->grad.release();
  p->work.release();
  p->part.release();
  delete p;
  return YY_OK;
}

extern "C" yy_status yy_proposal_num_params(yy_proposal p, int64_t* P) {
  if (!p || !P) return fail(YY_ERR_ARG, "yy_proposal_num_params: NULL argument");
  *P = p->P;
  return YY_OK;
}

extern "C" yy_status yy_proposal_get_params(yy_proposal p, float* params) {
  if (!p || !params) return fail(YY_ERR_ARG, "yy_proposal_get_params: NULL argument");
  YY_HIP(hipSetDevice(p->ctx->device));
  YY_HIP(hipMemcpyAsync(params, p->pf(), (size_t)p->P * sizeof(float), hipMemcpyDeviceToDevice, p->ctx->stream));
  return YY_OK;
}

extern "C" yy_status yy_proposal_set_params(yy_proposal p, const float* params) {
  if (!p || !params) return fail(YY_ERR_ARG, "yy_proposal_set_params: NULL argument");
  YY_HIP(hipSetDevice(p->ctx->device));
  const size_t bytes = (size_t)p->P * sizeof(float);
  hipStream_t st = p->ctx->stream;
  YY_HIP(hipMemcpyAsync(p->pf(), params, bytes, hipMemcpyDeviceToDevice, st));
  YY_HIP(hipMemsetAsync(p->adam_m.ptr, 0, bytes, st));
  YY_HIP(hipMemsetAsync(p->adam_v.ptr, 0, bytes, st));
  p->t = 0;
  return YY_OK;
}

extern "C" yy_status yy_proposal_forward(yy_proposal p, int32_t B, const double* xhat, float* out) {
  if (!p || !xhat || !out) return fail(YY_ERR_ARG, "yy_proposal_forward: NULL argument");
  if (B < 1 || B > (1 << 20)) return fail(YY_ERR_ARG, "yy_proposal_forward: B out of range");
  YY_HIP(hipSetDevice(p->ctx->device));
  Work w;
  yy_status s = work_for(p, B, w);
  if (s != YY_OK) return s;
  if ((s = forward(p, B, xhat, w)) != YY_OK) return s;
  YY_HIP(hipMemcpyAsync(out, w.O, (size_t)B * 2 * p->r * sizeof(float), hipMemcpyDeviceToDevice, p->ctx->stream));
  return YY_OK;
}

extern "C" yy_status yy_proposal_train_step(yy_proposal p, int32_t B, const double* xhat, const double* mu,
                                            const double* var, double R, double lr, int32_t update,
                                            double* loss, float* grad) {
  if (!p || !xhat || !mu || !var) return fail(YY_ERR_ARG, "yy_proposal_train_step: NULL argument");
  if (B < 1 || B > (1 << 20)) return fail(YY_ERR_ARG, "yy_proposal_train_step: B out of range");
  if (!(R > 0.0) || !std::isfinite(R)) return fail(YY_ERR_ARG, "yy_proposal_train_step: R must be positive");
  if (update && (!(lr > 0.0) || !std::isfinite(lr))) return fail(YY_ERR_ARG, "yy_proposal_train_step: bad lr");
  YY_HIP(hipSetDevice(p->ctx->device));
  hipStream_t st = p->ctx->stream;
  Work w;
  yy_status s = work_for(p, B, w);
  if (s != YY_OK) return s;
  const int64_t total = (int64_t)B * p->r;
  const int nb = (int)nblk(total);
  if ((s = p->part.ensure(((size_t)nb + 1) * sizeof(double))) != YY_OK) return s;
  if ((s = forward(p, B, xhat, w)) != YY_OK) return s;
  k_loss<<<nb, kBlock, 0, st>>>(B, p->r, w.O, xhat, mu, var, R, w.dO, p->part.as<double>());
  YY_LAUNCH_CHECK("k_loss");
  if (loss) {
    k_loss_final<<<1, 64, 0, st>>>(nb, total, p->part.as<double>(), loss);
    YY_LAUNCH_CHECK("k_loss_final");
  }
  float* g = p->grad.as<float>();
  if ((s = backward(p, B, w, g)) != YY_OK) return s;
  if (grad) YY_HIP(hipMemcpyAsync(grad, g, (size_t)p->P * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (update) {
    p->t += 1;
    const float bc1 = (float)(1.0 - std::pow(kB1, (double)p->t));
    const float bc2 = (float)(1.0 - std::pow(kB2, (double)p->t));
    k_adam<<<nblk(p->P), kBlock, 0, st>>>(p->P, p->pf(), g, p->adam_m.as<float>(), p->adam_v.as<float>(),
                                          (float)lr, bc1, bc2);
    YY_LAUNCH_CHECK("k_adam");
  }
  return YY_OK;
}

extern "C" yy_status yy_sample_moments(yy_ctx ctx, int64_t n, int32_t r, const double* x, const int64_t* idx,
                                       double* mean, double* var) {
  if (!ctx || !x || !idx || !mean || !var) return fail(YY_ERR_ARG, "yy_sample_moments: NULL argument");
  if (n < 1 || n > ((int64_t)1 << 32)) return fail(YY_ERR_ARG, "yy_sample_moments: n out of range");
  if (r < 1 || r > YY_MAX_R) return fail(YY_ERR_ARG, "yy_sample_moments: r out of range");
  YY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t nchunk = (n + kMomChunk - 1) / kMomChunk;
  yy_status s = ctx->red2.ensure((size_t)nchunk * r * sizeof(double));
  if (s != YY_OK) return s;
  double* part = ctx->red2.as<double>();
  dim3 grid(nblk(r), (unsigned)nchunk);
  k_mom_pass<<<grid, kBlock, 0, st>>>(n, r, x, idx, nullptr, part);
  YY_LAUNCH_CHECK("k_mom_pass");
  k_mom_reduce<<<nblk(r), kBlock, 0, st>>>(n, r, nchunk, part, mean);
  YY_LAUNCH_CHECK("k_mom_reduce");
  k_mom_pass<<<grid, kBlock, 0, st>>>(n, r, x, idx, mean, part);
  YY_LAUNCH_CHECK("k_mom_pass");
  k_mom_reduce<<<nblk(r), kBlock, 0, st>>>(n, r, nchunk, part, var);
  YY_LAUNCH_CHECK("k_mom_reduce");
  return YY_OK;
}
