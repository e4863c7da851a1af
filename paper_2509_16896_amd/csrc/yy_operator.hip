// yy_operator.hip -- the prediction as a stored operator (Sec. 10 offline /
// online split; Sec. 4.2 algorithm steps 2-3 and 5; Sec. 9 log domain).
//
// Offline (once per node set): every kernel value of the node set is stored,
// per scale, as a base-2 exponent without the weights,
//   E[s][i][j] = -kap_s |x_i - x_j - tau_s f_j|^2   (push form; pull form
//                -kap_s |x_i - tau_s f_i - x_j|^2),   kap_s = log2(e) / (2 q tau_s),
// by FP32 direct differences (the arithmetic of the vector-ALU pairwise form;
// the self pair from the FP64 norm |tau_s f_i|^2), FP32, rows padded to a
// multiple of 64 sources with -inf.  With general process noise the node set
// is whitened first, as in yy_propagate.
// Online (every step): the paper multiplies the stored matrix by the weight
// vector; here, in the log domain, every (scale, target) row takes the
// log-sum-exp of E[s][i][:] + lw2 (the weights in base 2 relative to their
// maximum): one wavefront streams one row (16-byte loads), so the step reads
// S n^2 x 4 bytes once and is bound by memory bandwidth (HBM, or the
// last-level cache while the operator fits in it).  The FP64 combination of
// the scales, the constants, the identity term and the clamp are those of
// yy_propagate (k_combine).
#include <algorithm>
#include <cmath>

#include "yy_common.h"
#include "yy_internal.h"

struct yy_operator_s {
  yy_ctx ctx = nullptr;
  int64_t n = 0, ld = 0;       // nodes, row length (n rounded up to 64)
  int32_t S = 0;
  yy::DevBuf E;                // float [S][n][ld]
  yy::DevBuf bnd, div, scal;   // int [n], double [n] (pull form), double [8]
  yy::DevBuf lw2;              // float [ld], -inf beyond n
  yy::DevBuf part;             // float2 [S][n]
  yy::DevBuf lw0;              // double [n] zeros (the weights of the build's plan)
  yy::DevBuf out0;             // double [n] (the build plan's output slot, never written)
  yy::CombineArgs cb{};        // the combination's constants, from the build
};

namespace yy {

constexpr int kOT = 64;   // targets and sources per build tile

struct OpScales {
  float kap[YY_MAX_SCALES], tau[YY_MAX_SCALES];
  double kapd[YY_MAX_SCALES], taud[YY_MAX_SCALES];
};

template <int S, int KC, bool PULL>
__global__ void __launch_bounds__(256) k_op_build(PairArgs a, OpScales sc, int64_t ld, float* __restrict__ E) {
  __shared__ float sxi[KC][kOT + 4];
  __shared__ float sxj[KC][kOT + 4];
  __shared__ float sf[KC][kOT + 4];
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int64_t n = a.n;
  const int64_t i0 = (int64_t)blockIdx.y * kOT, j0 = (int64_t)blockIdx.x * kOT;
  float acc[4][4][S];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int s = 0; s < S; ++s) acc[p][q][s] = 0.f;
  for (int k0 = 0; k0 < a.r; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < kOT * KC; e += 256) {
      const int row = e / KC, kk = e % KC;
      const int k = k0 + kk;
      const int64_t gi = i0 + row, gj = j0 + row;
      const bool vi = gi < n && k < a.r, vj = gj < n && k < a.r;
      sxi[kk][row] = vi ? a.xc[(size_t)gi * a.rp + k] : 0.f;
      sxj[kk][row] = vj ? a.xc[(size_t)gj * a.rp + k] : 0.f;
      if (PULL) sf[kk][row] = vi ? a.f[(size_t)gi * a.rp + k] : 0.f;
      else sf[kk][row] = vj ? a.f[(size_t)gj * a.rp + k] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const float4 xi = *reinterpret_cast<const float4*>(&sxi[kk][ti * 4]);
      const float4 xj = *reinterpret_cast<const float4*>(&sxj[kk][tj * 4]);
      const float4 fv = *reinterpret_cast<const float4*>(&sf[kk][(PULL ? ti : tj) * 4]);
      const float xia[4] = {xi.x, xi.y, xi.z, xi.w};
      const float xja[4] = {xj.x, xj.y, xj.z, xj.w};
      const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float d = xia[p] - xja[q];
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const float e = fmaf(-sc.tau[s], fa[PULL ? p : q], d);
            acc[p][q][s] = fmaf(e, e, acc[p][q][s]);
          }
        }
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t gi = i0 + ti * 4 + p;
    if (gi >= n) continue;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gj = j0 + tj * 4 + q;
        float e = -sc.kap[s] * acc[p][q][s];
        if (gj == gi) e = -(float)(sc.kapd[s] * sc.taud[s] * sc.taud[s] * a.node[n + gi]);   // |tau f_i|^2
        if (gj >= n) e = -INFINITY;
        v[q] = e;
      }
      *reinterpret_cast<float4*>(E + ((size_t)s * n + gi) * ld + j0 + tj * 4) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

template <int S, bool PULL>
static void launch_build_kc(hipStream_t st, dim3 grid, const PairArgs& a, const OpScales& sc, int64_t ld, float* E) {
  if (a.r <= 4) k_op_build<S, 4, PULL><<<grid, 256, 0, st>>>(a, sc, ld, E);
  else if (a.r <= 8) k_op_build<S, 8, PULL><<<grid, 256, 0, st>>>(a, sc, ld, E);
  else k_op_build<S, 16, PULL><<<grid, 256, 0, st>>>(a, sc, ld, E);
}

template <int S>
static void launch_build_s(hipStream_t st, dim3 grid, const PairArgs& a, const OpScales& sc, int64_t ld, float* E) {
  if (a.pull) launch_build_kc<S, true>(st, grid, a, sc, ld, E);
  else launch_build_kc<S, false>(st, grid, a, sc, ld, E);
}

__global__ void __launch_bounds__(kBlock) k_fill_f32(int64_t count, float v, float* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = v;
}

// One wavefront per (scale, target) row: (max, sum) in base 2 of E[s][i][:] + lw2.
__global__ void __launch_bounds__(kBlock) k_op_apply(int64_t n, int32_t S, int64_t ld, const float* __restrict__ E,
                                                     const float* __restrict__ lw2, float2* __restrict__ part) {
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;   // s * n + i
  const int lane = threadIdx.x & 63;
  if (row >= (int64_t)S * n) return;
  const float4* e4 = reinterpret_cast<const float4*>(E + (size_t)row * ld);
  const float4* w4 = reinterpret_cast<const float4*>(lw2);
  float M = -INFINITY, Sum = 0.f;
  for (int64_t q = lane; q < ld / 4; q += 64) {
    const float4 e = e4[q], w = w4[q];
    const float v[4] = {e.x + w.x, e.y + w.y, e.z + w.z, e.w + w.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (v[u] == -INFINITY) continue;
      if (v[u] > M) {
        Sum = Sum * __builtin_amdgcn_exp2f(M - v[u]) + 1.f;
        M = v[u];
      } else {
        Sum += __builtin_amdgcn_exp2f(v[u] - M);
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float mo = __shfl_xor(M, off, 64);
    const float so = __shfl_xor(Sum, off, 64);
    lse2_merge(M, Sum, mo, so);
  }
  if (lane == 0) part[row] = make_float2(M, Sum);
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_operator_build(yy_ctx ctx, const yy_model* model, const yy_scales* scales, int64_t n,
                                       const double* x, uint64_t node_version, const double* box_lo,
                                       const double* box_hi, double dt, yy_operator* inout) {
  if (!ctx || !inout) return fail(YY_ERR_ARG, "yy_operator_build: NULL argument");
  if (n < 1) return fail(YY_ERR_ARG, "yy_operator_build: n < 1");
  if (!scales || scales->S < 1 || scales->S > YY_MAX_SCALES) return fail(YY_ERR_ARG, "yy_operator_build: bad scales");
  YY_HIP(hipSetDevice(ctx->device));
  yy_operator op = *inout;
  const bool fresh = op == nullptr;
  if (fresh) {
    op = new (std::nothrow) yy_operator_s();
    if (!op) return fail(YY_ERR_ALLOC, "yy_operator_build: out of host memory");
    op->ctx = ctx;
  } else if (op->ctx != ctx) {
    return fail(YY_ERR_ARG, "yy_operator_build: the operator belongs to another context");
  }
  auto bail = [&](yy_status st) {
    if (fresh) {
      op->E.release(); op->bnd.release(); op->div.release(); op->scal.release(); op->lw2.release();
      op->part.release(); op->lw0.release(); op->out0.release();
      delete op;
    }
    return st;
  };
  const int32_t S = scales->S;
  const int64_t ld = ((n + 63) / 64) * 64;
  yy_status st;
  if ((st = op->lw0.ensure((size_t)n * sizeof(double))) != YY_OK) return bail(st);
  if ((st = op->out0.ensure((size_t)n * sizeof(double))) != YY_OK) return bail(st);
  hipError_t he = hipMemsetAsync(op->lw0.ptr, 0, (size_t)n * sizeof(double), ctx->stream);
  if (he != hipSuccess) return bail(hip_fail(he, "hipMemsetAsync(lw0)"));
  // the plan of a plain FP32 propagation: prepared (and, with general noise, whitened) node set,
  // divergence (pull form), constants of the combination
  PropPlan plan;
  if ((st = propagate_begin(ctx, model, scales, YY_PREC_FP32, n, x, node_version, box_lo, box_hi, dt,
                            op->lw0.as<double>(), op->out0.as<double>(), 1, plan, false)) != YY_OK)
    return bail(st);
  const size_t ebytes = (size_t)S * n * ld * sizeof(float);
  if ((st = op->E.ensure(ebytes)) != YY_OK) return bail(st);
  if ((st = op->bnd.ensure((size_t)n * sizeof(int))) != YY_OK) return bail(st);
  if ((st = op->div.ensure((size_t)n * sizeof(double))) != YY_OK) return bail(st);
  if ((st = op->scal.ensure(8 * sizeof(double))) != YY_OK) return bail(st);
  if ((st = op->lw2.ensure((size_t)ld * sizeof(float))) != YY_OK) return bail(st);
  if ((st = op->part.ensure((size_t)S * n * sizeof(float2))) != YY_OK) return bail(st);
  const Prepared& P = ctx->prep;
  // the operator keeps its own copies of what the online stage reads
  if ((he = hipMemcpyAsync(op->bnd.ptr, P.bnd.ptr, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream)) !=
          hipSuccess ||
      (he = hipMemcpyAsync(op->scal.ptr, P.scal.ptr, 8 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream)) !=
          hipSuccess)
    return bail(hip_fail(he, "hipMemcpyAsync(operator)"));
  if (plan.a.pull &&
      (he = hipMemcpyAsync(op->div.ptr, P.div.ptr, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream)) !=
          hipSuccess)
    return bail(hip_fail(he, "hipMemcpyAsync(div)"));
  k_fill_f32<<<(unsigned)((ld + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(ld, -INFINITY, op->lw2.as<float>());
  YY_LAUNCH_CHECK("k_fill_f32");
  OpScales sc{};
  for (int s = 0; s < S; ++s) {
    sc.kap[s] = plan.a.kap2[s];
    sc.tau[s] = plan.a.tau[s];
    sc.kapd[s] = plan.kapd[s];
    sc.taud[s] = plan.taud[s];
  }
  dim3 grid((unsigned)(ld / kOT), (unsigned)((n + kOT - 1) / kOT));
  float* E = op->E.as<float>();
  switch (S) {
    case 1: launch_build_s<1>(ctx->stream, grid, plan.a, sc, ld, E); break;
    case 2: launch_build_s<2>(ctx->stream, grid, plan.a, sc, ld, E); break;
    case 3: launch_build_s<3>(ctx->stream, grid, plan.a, sc, ld, E); break;
    case 4: launch_build_s<4>(ctx->stream, grid, plan.a, sc, ld, E); break;
    case 5: launch_build_s<5>(ctx->stream, grid, plan.a, sc, ld, E); break;
    default: launch_build_s<6>(ctx->stream, grid, plan.a, sc, ld, E); break;
  }
  YY_LAUNCH_CHECK("k_op_build");
  op->n = n;
  op->ld = ld;
  op->S = S;
  op->cb = plan.cb;
  op->cb.part = op->part.as<float2>();
  op->cb.nsplit = 1;
  op->cb.bnd = op->bnd.as<int>();
  op->cb.scal = op->scal.as<double>();
  op->cb.div = plan.a.pull ? op->div.as<double>() : nullptr;
  op->cb.defer = nullptr;
  op->cb.j_per_split = n;
  *inout = op;
  return YY_OK;
}

extern "C" yy_status yy_operator_apply(yy_operator op, const double* logw_in, double* logw_out) {
  if (!op) return fail(YY_ERR_ARG, "yy_operator_apply: NULL operator");
  if (!logw_in || !logw_out) return fail(YY_ERR_ARG, "yy_operator_apply: NULL array");
  if (logw_in == logw_out) return fail(YY_ERR_ARG, "yy_operator_apply: logw_in and logw_out alias");
  yy_ctx ctx = op->ctx;
  YY_HIP(hipSetDevice(ctx->device));
  yy_status st;
  double* lref = nullptr;
  if ((st = source_weights(ctx, op->n, logw_in, op->bnd.as<int>(), op->lw2.as<float>(), &lref)) != YY_OK) return st;
  if ((st = timing_begin(ctx)) != YY_OK) return st;
  const int64_t rows = (int64_t)op->S * op->n;
  k_op_apply<<<(unsigned)((rows * 64 + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
      op->n, op->S, op->ld, op->E.as<float>(), op->lw2.as<float>(), op->part.as<float2>());
  YY_LAUNCH_CHECK("k_op_apply");
  if ((st = timing_end(ctx)) != YY_OK) return st;
  CombineArgs cb = op->cb;
  cb.lref = lref;
  cb.logw_in = logw_in;
  cb.logw_out = logw_out;
  cb.flags = ctx->d_flags;
  cb.nclamped = ctx->d_nclamped;
  return launch_combine(ctx->stream, cb);
}

extern "C" yy_status yy_operator_info(yy_operator op, int64_t* n, int32_t* S, int64_t* bytes) {
  if (!op) return fail(YY_ERR_ARG, "yy_operator_info: NULL operator");
  if (n) *n = op->n;
  if (S) *S = op->S;
  if (bytes) *bytes = (int64_t)op->S * op->n * op->ld * (int64_t)sizeof(float);
  return YY_OK;
}

extern "C" yy_status yy_operator_destroy(yy_operator op) {
  if (!op) return YY_OK;
  (void)hipSetDevice(op->ctx->device);
  if (op->ctx->stream) (void)hipStreamSynchronize(op->ctx->stream);
  op->E.release();
  op->bnd.release();
  op->div.release();
  op->scal.release();
  op->lw2.release();
  op->part.release();
  op->lw0.release();
  op->out0.release();
  delete op;
  return YY_OK;
}
