// yy_noise.hip -- general noise coefficients (Sec. 7, Table tab:generalformulas):
// dx = f dt + U dV, dy = h dt + V dW with a = U U^T and b = V V^T, invertible
// or singular (then a^+, b^+ and det_+ replace the inverse and determinant).
//
// The quadratic forms of the kernel and of the correction are sums of squares
// in whitened coordinates: with a = Q diag(lam) Q^T and W = diag(lam_+^-1/2) Q_+^T
// (k x r, the rows of the positive eigenvalues), W^T W = a^+ and
//   |d|^2_{a^+} = |W d|^2,
// so the node set is whitened once per node version (x~ = W (x - c),
// f~ = W f(x), FP64 GEMMs) and the pairwise kernels run unchanged on x~, f~
// with unit variance; the Gaussian constant becomes
// -(r/2) log(2 pi tau) - (1/2) log det_+ a (the table's constant in both cases).
// The correction h^T b^+ dy - dt/2 h^T b^+ h = z . w - dt/2 |z|^2 with
// z = W_b h(x_i) (a GEMM over the nodes) and w = W_b dy.
//
// The eigen-decomposition runs once, on the host, when the noise object is
// created (cyclic Jacobi rotations on the symmetric matrix).
#include <algorithm>
#include <cmath>
#include <vector>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

// ---------------------------------------------------------------------------
// Host: eigen-decomposition of a symmetric matrix by cyclic Jacobi rotations.
// Each rotation zeroes one off-diagonal entry (angle from the 2x2 symmetric
// eigenproblem, the smaller root of t^2 + 2 theta t - 1 = 0 for stability);
// sweeps repeat until the off-diagonal mass is below 1e-30 of the total.
static void jacobi_eigen(int N, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Q) {
  Q.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) Q[(size_t)i * N + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * N + j]; };
  double total = 0.0;
  for (size_t e = 0; e < A.size(); ++e) total += A[e] * A[e];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) off += 2.0 * at(i, j) * at(i, j);
    if (!(off > 1e-30 * total)) break;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q) {
        const double apq = at(p, q);
        if (apq == 0.0) continue;
        const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A <- R^T A R on rows/columns p, q
        for (int k = 0; k < N; ++k) {
          const double akp = at(k, p), akq = at(k, q);
          at(k, p) = c * akp - s * akq;
          at(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = at(p, k), aqk = at(q, k);
          at(p, k) = c * apk - s * aqk;
          at(q, k) = s * apk + c * aqk;
        }
        at(p, q) = at(q, p) = 0.0;
        for (int k = 0; k < N; ++k) {
          double* row = &Q[(size_t)k * N];
          const double qkp = row[p], qkq = row[q];
          row[p] = c * qkp - s * qkq;
          row[q] = s * qkp + c * qkq;
        }
      }
  }
  lam.resize(N);
  for (int i = 0; i < N; ++i) lam[i] = at(i, i);
}

// Whitening rows W (k x N, row-major) and log det_+ of M = C C^T (C: N x N row-major).
static void whitening(int N, const double* C, std::vector<double>& W, int& rank, double& logdet) {
  std::vector<double> M((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double acc = 0.0;
      for (int l = 0; l < N; ++l) acc += C[(size_t)i * N + l] * C[(size_t)j * N + l];
      M[(size_t)i * N + j] = acc;
    }
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      const double v = 0.5 * (M[(size_t)i * N + j] + M[(size_t)j * N + i]);
      M[(size_t)i * N + j] = M[(size_t)j * N + i] = v;
    }
  std::vector<double> lam, Q;
  jacobi_eigen(N, M, lam, Q);
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, v);
  rank = 0;
  logdet = 0.0;
  W.clear();
  for (int e = 0; e < N; ++e) {
    if (!(lam[e] > kNoisePinvRtol * lmax)) continue;   // the pseudo-inverse drops this eigenvalue
    ++rank;
    logdet += std::log(lam[e]);
    const double sc = 1.0 / std::sqrt(lam[e]);
    for (int j = 0; j < N; ++j) W.push_back(sc * Q[(size_t)j * N + e]);
  }
}

// ---------------------------------------------------------------------------
// Device: C = A B^T in FP64 (A: M x K, B: N x K, C: M x N, all row-major with
// the given leading dimensions), 64 x 64 tiles, K in chunks of 16 through LDS,
// each thread a 4 x 4 block, products summed in increasing k.
constexpr int kGT = 64, kGK = 16;
__global__ void __launch_bounds__(256) k_gemm_nt_f64(int64_t M, int32_t N, int32_t K, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                     double* __restrict__ C, int64_t ldc) {
  __shared__ double As[kGK][kGT + 1];
  __shared__ double Bs[kGK][kGT + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * kGT;
  const int32_t n0 = blockIdx.y * kGT;
  double acc[4][4] = {};
  for (int32_t k0 = 0; k0 < K; k0 += kGK) {
    for (int e = tid; e < kGT * kGK; e += 256) {
      const int row = e / kGK, kk = e % kGK;
      const int64_t gm = m0 + row;
      const int32_t gn = n0 + row, gk = k0 + kk;
      As[kk][row] = (gm < M && gk < K) ? A[gm * lda + gk] : 0.0;
      Bs[kk][row] = (gn < N && gk < K) ? B[(int64_t)gn * ldb + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty * 4 + u];
        b[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t gm = m0 + ty * 4 + u;
    if (gm >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int32_t gn = n0 + tx * 4 + v;
      if (gn < N) C[gm * ldc + gn] = acc[u][v];
    }
  }
}

static yy_status gemm_nt(hipStream_t st, int64_t M, int32_t N, int32_t K, const double* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc) {
  if (M == 0 || N == 0) return YY_OK;
  dim3 grid((unsigned)((M + kGT - 1) / kGT), (unsigned)((N + kGT - 1) / kGT));
  k_gemm_nt_f64<<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc);
  YY_LAUNCH_CHECK("k_gemm_nt_f64");
  return YY_OK;
}

// Centred coordinates, drift values and boundary flags of the nodes in the
// original coordinates (one thread per node and coordinate, a block row per node).
__global__ void __launch_bounds__(kBlock) k_whiten_inputs(int64_t n, int32_t r, int32_t drift,
                                                          const double* __restrict__ A, const double* __restrict__ x,
                                                          const double* __restrict__ lo, const double* __restrict__ hi,
                                                          double* __restrict__ xc, double* __restrict__ fx,
                                                          int* __restrict__ bnd) {
  __shared__ int sb;
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  if (threadIdx.x == 0) sb = 0;
  __syncthreads();
  const double* xi = x + (size_t)i * r;
  int b = 0;
  for (int32_t k = threadIdx.x; k < r; k += kBlock) {
    const double xv = xi[k];
    xc[(size_t)i * r + k] = xv - 0.5 * (lo[k] + hi[k]);
    b |= (fabs(xv - lo[k]) <= kBoundaryTol) || (fabs(hi[k] - xv) <= kBoundaryTol);
    double fv = 0.0;
    if (drift == YY_F_COS) {
      fv = cos(xv);
    } else if (drift == YY_F_PAPER_SINMIX) {
      const double xn = k + 1 < r ? xi[k + 1] : 0.0;
      fv = sin(xv) * (-0.5 * xv + 0.1 * xn) + sin(2.0 * xv) * (-0.3 * xv + 0.3 * xn);
    } else if (drift == YY_F_LINEAR) {
      const double* Ak = A + (size_t)k * r;
      double acc = 0.0;
      for (int32_t l = 0; l < r; ++l) acc = fma(Ak[l], xi[l], acc);
      fv = acc;
    }
    fx[(size_t)i * r + k] = fv;
  }
  if (b) atomicOr(&sb, 1);
  __syncthreads();
  if (threadIdx.x == 0) bnd[i] = sb;
}

// h(x_i) for every node, row-major [n x m].
__global__ void __launch_bounds__(kBlock) k_obs_rows(int64_t n, int32_t r, int32_t m, int32_t obs,
                                                     const double* __restrict__ H, double h_shift,
                                                     const double* __restrict__ x, double* __restrict__ hx) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const double* xi = x + (size_t)i * r;
  for (int32_t k = threadIdx.x; k < m; k += kBlock) {
    double v;
    if (obs == YY_H_IDENTITY) {
      v = xi[k];
    } else if (obs == YY_H_CUBE) {
      const double t = xi[k] - h_shift;
      v = t * t * t;
    } else {
      const double* Hk = H + (size_t)k * r;
      double acc = 0.0;
      for (int32_t l = 0; l < r; ++l) acc = fma(Hk[l], xi[l], acc);
      v = acc;
    }
    hx[(size_t)i * m + k] = v;
  }
}

// w = W_b dy (one block).
__global__ void __launch_bounds__(kBlock) k_white_dy(int32_t kb, int32_t m, const double* __restrict__ Wb,
                                                     const double* __restrict__ dy, double* __restrict__ w) {
  for (int32_t e = threadIdx.x; e < kb; e += kBlock) {
    double acc = 0.0;
    for (int32_t l = 0; l < m; ++l) acc = fma(Wb[(size_t)e * m + l], dy[l], acc);
    w[e] = acc;
  }
}

// logw_i += z_i . w - dt/2 |z_i|^2 (a wave per node, fixed-order reduction).
__global__ void __launch_bounds__(kBlock) k_loglik_white(int64_t n, int32_t kb, const double* __restrict__ z,
                                                         const double* __restrict__ w, double dt,
                                                         double* __restrict__ logw) {
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double lin = 0.0, quad = 0.0;
  for (int32_t e = lane; e < kb; e += 64) {
    const double v = z[(size_t)i * kb + e];
    lin = fma(v, w[e], lin);
    quad = fma(v, v, quad);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lin += __shfl_xor(lin, off, 64);
    quad += __shfl_xor(quad, off, 64);
  }
  if (lane == 0 && logw[i] != -INFINITY) logw[i] += lin - 0.5 * dt * quad;
}

// ---------------------------------------------------------------------------
yy_status noise_whiten_nodes(yy_ctx ctx, const yy_model* m, int64_t n, const double* x, const double* lo,
                             const double* hi, WhiteNodes& out) {
  const yy_noise nz = m->noise;
  const int32_t r = m->r, k = nz->rank_a;
  Prepared& P = ctx->prep;
  yy_status st;
  if ((st = P.wtmp.ensure((size_t)2 * n * r * sizeof(double))) != YY_OK) return st;
  if ((st = P.wnodes.ensure((size_t)2 * n * k * sizeof(double))) != YY_OK) return st;
  if ((st = P.wbnd.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(int))) != YY_OK) return st;
  double* xc = P.wtmp.as<double>();
  double* fx = xc + (size_t)n * r;
  double* xw = P.wnodes.as<double>();
  double* fw = xw + (size_t)n * k;
  k_whiten_inputs<<<(unsigned)n, kBlock, 0, ctx->stream>>>(n, r, m->drift, m->A, x, lo, hi, xc, fx,
                                                           P.wbnd.as<int>());
  YY_LAUNCH_CHECK("k_whiten_inputs");
  const double* Wa = nz->Wa.as<double>();
  if ((st = gemm_nt(ctx->stream, n, k, r, xc, r, Wa, r, xw, k)) != YY_OK) return st;
  if ((st = gemm_nt(ctx->stream, n, k, r, fx, r, Wa, r, fw, k)) != YY_OK) return st;
  out.x = xw;
  out.f = fw;
  out.bnd = P.wbnd.as<int>();
  out.zeros = nz->zeros.as<double>();
  out.k = k;
  return YY_OK;
}

yy_status noise_loglik(yy_ctx ctx, const yy_model* m, int64_t n, const double* x, const double* dy, double dt,
                       double* logw) {
  const yy_noise nz = m->noise;
  const int32_t kb = nz->rank_b, mm = m->m;
  yy_status st;
  if ((st = ctx->obsw.ensure(((size_t)n * mm + (size_t)n * kb + kb) * sizeof(double))) != YY_OK) return st;
  double* hx = ctx->obsw.as<double>();
  double* z = hx + (size_t)n * mm;
  double* w = z + (size_t)n * kb;
  k_obs_rows<<<(unsigned)n, kBlock, 0, ctx->stream>>>(n, m->r, mm, m->obs, m->H, m->h_shift, x, hx);
  YY_LAUNCH_CHECK("k_obs_rows");
  const double* Wb = nz->Wb.as<double>();
  k_white_dy<<<1, kBlock, 0, ctx->stream>>>(kb, mm, Wb, dy, w);
  YY_LAUNCH_CHECK("k_white_dy");
  if ((st = gemm_nt(ctx->stream, n, kb, mm, hx, mm, Wb, mm, z, kb)) != YY_OK) return st;
  const int64_t blocks = (n * 64 + kBlock - 1) / kBlock;
  k_loglik_white<<<(unsigned)blocks, kBlock, 0, ctx->stream>>>(n, kb, z, w, dt, logw);
  YY_LAUNCH_CHECK("k_loglik_white");
  return YY_OK;
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_noise_create(yy_ctx ctx, int32_t r, const double* U, int32_t m, const double* V,
                                     yy_noise* out) {
  if (!ctx || !out) return fail(YY_ERR_ARG, "yy_noise_create: NULL argument");
  *out = nullptr;
  if (r < 1 || r > YY_MAX_R || m < 1 || m > YY_MAX_R) return fail(YY_ERR_ARG, "yy_noise_create: r or m out of range");
  if (!U && !V) return fail(YY_ERR_ARG, "yy_noise_create: neither U nor V given");
  YY_HIP(hipSetDevice(ctx->device));
  yy_noise nz = new (std::nothrow) yy_noise_s();
  if (!nz) return fail(YY_ERR_ALLOC, "yy_noise_create: out of host memory");
  nz->ctx = ctx;
  nz->r = r;
  nz->m = m;
  yy_status st = YY_OK;
  auto upload = [&](DevBuf& buf, const std::vector<double>& h) -> yy_status {
    yy_status s2 = buf.ensure(std::max<size_t>(h.size(), 1) * sizeof(double));
    if (s2 != YY_OK) return s2;
    if (!h.empty()) {
      hipError_t e = hipMemcpy(buf.ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpy(noise)");
    }
    return YY_OK;
  };
  if (U) {
    std::vector<double> W;
    whitening(r, U, W, nz->rank_a, nz->logdet_a);
    if (nz->rank_a == 0) st = fail(YY_ERR_ARG, "yy_noise_create: a = U U^T is zero");
    if (st == YY_OK) st = upload(nz->Wa, W);
  }
  if (st == YY_OK && V) {
    std::vector<double> W;
    whitening(m, V, W, nz->rank_b, nz->logdet_b);
    if (nz->rank_b == 0) st = fail(YY_ERR_ARG, "yy_noise_create: b = V V^T is zero");
    if (st == YY_OK) st = upload(nz->Wb, W);
  }
  if (st == YY_OK) st = upload(nz->zeros, std::vector<double>((size_t)std::max(r, m), 0.0));
  if (st != YY_OK) {
    nz->Wa.release();
    nz->Wb.release();
    nz->zeros.release();
    delete nz;
    return st;
  }
  *out = nz;
  return YY_OK;
}

extern "C" yy_status yy_noise_destroy(yy_noise nz) {
  if (!nz) return YY_OK;
  (void)hipSetDevice(nz->ctx->device);
  if (nz->ctx->stream) (void)hipStreamSynchronize(nz->ctx->stream);
  nz->Wa.release();
  nz->Wb.release();
  nz->zeros.release();
  delete nz;
  return YY_OK;
}

extern "C" yy_status yy_noise_info(yy_noise nz, int32_t* rank_a, double* logdet_a, int32_t* rank_b,
                                   double* logdet_b) {
  if (!nz) return fail(YY_ERR_ARG, "yy_noise_info: NULL noise");
  if (rank_a) *rank_a = nz->rank_a;
  if (logdet_a) *logdet_a = nz->logdet_a;
  if (rank_b) *rank_b = nz->rank_b;
  if (logdet_b) *logdet_b = nz->logdet_b;
  return YY_OK;
}
