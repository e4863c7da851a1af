// yy_restart.hip -- the local resample-restart (Sec. 6): integer systematic
// resampling of the normalised weights, a new box [mean - R, mean + R]^r,
// the pre-generated reference codes mapped to that box, and the restart prior
// (the initial density re-centred at the estimate).
#include <algorithm>
#include <cmath>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

static const uint64_t kDomainResample = 2ULL;

// SplitMix64 (Steele, Lea, Flood 2014) at counter position `counter` of stream `seed`.
__device__ inline uint64_t d_sm64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint64_t h_sm64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Integer weights W_i = floor(w_i 2^53) and their inclusive prefix sums within
// each block of kBlock elements; block totals go to `tot`.
__device__ __forceinline__ void k_rs_local_body(int64_t n, const double* __restrict__ w,
                                                     unsigned long long* __restrict__ C,
                                                     unsigned long long* __restrict__ tot, int bx_, int gx_) {
  __shared__ unsigned long long s[kBlock];
  const int64_t i = (int64_t)bx_ * kBlock + threadIdx.x;
  unsigned long long v = 0;
  if (i < n) {
    const double wi = w[i] > 0.0 ? w[i] : 0.0;
    v = (unsigned long long)floor(wi * 0x1p53);
  }
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {  // Hillis-Steele inclusive scan
    unsigned long long t = threadIdx.x >= off ? s[threadIdx.x - off] : 0ULL;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) C[i] = s[threadIdx.x];
  if (threadIdx.x == kBlock - 1) tot[bx_] = s[kBlock - 1];
}

__global__ void __launch_bounds__(kBlock) k_rs_local_batch(const rs_local_args* __restrict__ A,
                                                           const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const rs_local_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_rs_local_body(a.n, a.w, a.C, a.tot, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// Exclusive offsets of the block totals (one block; integer sums, so any
// order of the additions gives the same offsets): 256 totals at a time, a
// scan in LDS, the running carry across the rounds.
__device__ __forceinline__ void k_rs_offsets_body(int nb, unsigned long long* __restrict__ tot, int bx_, int gx_) {
  __shared__ unsigned long long s[kBlock];
  if (bx_ != 0) return;
  const int tid = threadIdx.x;
  unsigned long long carry = 0;
  for (int base = 0; base < nb; base += kBlock) {
    const int b = base + tid;
    const unsigned long long v = b < nb ? tot[b] : 0ULL;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      const unsigned long long t = tid >= off ? s[tid - off] : 0ULL;
      __syncthreads();
      s[tid] += t;
      __syncthreads();
    }
    if (b < nb) tot[b] = carry + s[tid] - v;
    carry += s[kBlock - 1];
    __syncthreads();
  }
  if (tid == 0) tot[nb] = carry;  // W
}

__global__ void __launch_bounds__(kBlock) k_rs_offsets(int nb, unsigned long long* __restrict__ tot) {
  k_rs_offsets_body(nb, tot, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_rs_offsets_batch(const rs_offsets_args* __restrict__ A,
                                                             const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const rs_offsets_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_rs_offsets_body(a.nb, a.tot, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


__device__ __forceinline__ void k_rs_add_body(int64_t n, const unsigned long long* __restrict__ tot,
                                                   unsigned long long* __restrict__ C, int bx_, int gx_) {
  const int64_t i = (int64_t)bx_ * kBlock + threadIdx.x;
  if (i < n) C[i] += tot[bx_];
}

__global__ void __launch_bounds__(kBlock) k_rs_add(int64_t n, const unsigned long long* __restrict__ tot,
                                                   unsigned long long* __restrict__ C) {
  k_rs_add_body(n, tot, C, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_rs_add_batch(const rs_add_args* __restrict__ A,
                                                         const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const rs_add_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_rs_add_body(a.n, a.tot, a.C, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// P_t = floor((t 2^32 + U) W / (n 2^32)); idx[t] = min{i : C_i > P_t}.
// The 119-bit product is formed from 64-bit halves; the quotient is taken as
// floor(floor(A W / 2^32) / n) with a 96-by-32-bit long division.
__device__ __forceinline__ void k_rs_search_body(int64_t n, int nb,
                                                      const unsigned long long* __restrict__ tot,
                                                      const unsigned long long* __restrict__ C,
                                                      uint64_t U, int64_t* __restrict__ idx,
                                                      uint32_t* __restrict__ flags, int bx_, int gx_) {
  const int64_t t = (int64_t)bx_ * kBlock + threadIdx.x;
  const unsigned long long W = tot[nb];
  if (W == 0ULL) {
    if (t == 0) atomicOr(flags, YY_FLAG_RESAMPLE_ZERO);
    return;
  }
  if (t >= n) return;
  const uint64_t A = ((uint64_t)t << 32) + U;
  const uint64_t lo = A * W;
  const uint64_t hi = __umul64hi(A, W);
  // X = (hi:lo) >> 32, at most 86 bits: three 32-bit digits x2 x1 x0.
  const uint64_t x0 = (lo >> 32) & 0xFFFFFFFFULL;
  const uint64_t x1 = hi & 0xFFFFFFFFULL;
  const uint64_t x2 = hi >> 32;
  const uint64_t d = (uint64_t)n;
  // P < W <= 2^54, so the top quotient digit x2 / n is zero and the
  // remainders below stay under n < 2^32.
  uint64_t rem = x2 % d;
  uint64_t cur = (rem << 32) | x1;
  const uint64_t q1 = cur / d;
  rem = cur % d;
  cur = (rem << 32) | x0;
  const uint64_t q0 = cur / d;
  const uint64_t P = (q1 << 32) + q0;
  int64_t lo_i = 0, hi_i = n - 1;  // C[n-1] = W > P, so the answer exists
  while (lo_i < hi_i) {
    const int64_t mid = (lo_i + hi_i) >> 1;
    if (C[mid] > P) hi_i = mid;
    else lo_i = mid + 1;
  }
  idx[t] = lo_i;
}

__global__ void __launch_bounds__(kBlock) k_rs_search(int64_t n, int nb,
                                                      const unsigned long long* __restrict__ tot,
                                                      const unsigned long long* __restrict__ C,
                                                      uint64_t U, int64_t* __restrict__ idx,
                                                      uint32_t* __restrict__ flags) {
  k_rs_search_body(n, nb, tot, C, U, idx, flags, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_rs_search_batch(const rs_search_args* __restrict__ A,
                                                            const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const rs_search_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_rs_search_body(a.n, a.nb, a.tot, a.C, a.kstep ? d_sm64(a.key, (uint64_t)*a.kstep) >> 32 : a.U, a.idx,
                   a.flags, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// The plain box [mean - R, mean + R]^r.
__device__ __forceinline__ void k_box_plain_body(int32_t r, double R, const double* __restrict__ mean,
                                                      double* __restrict__ box_lo,
                                                      double* __restrict__ box_hi, int bx_, int gx_) {
  const int d = bx_ * kBlock + threadIdx.x;
  if (d >= r) return;
  box_lo[d] = __dsub_rn(mean[d], R);
  box_hi[d] = __dadd_rn(mean[d], R);
}

__global__ void __launch_bounds__(kBlock) k_box_plain(int32_t r, double R, const double* __restrict__ mean,
                                                      double* __restrict__ box_lo, double* __restrict__ box_hi) {
  k_box_plain_body(r, R, mean, box_lo, box_hi, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_box_plain_batch(const box_plain_args* __restrict__ A,
                                                            const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const box_plain_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_box_plain_body(a.r, a.R, a.mean, a.box_lo, a.box_hi, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// Nodes and prior in the box [box_lo, box_hi].  One wavefront per node; the
// centre and half-width are recomputed per coordinate exactly as the node
// map defines them (no fused multiply-add).  With `only_if` set the kernel
// runs only when *only_if is non-zero (the learned restart's fallback).
__device__ __forceinline__ void k_restart_nodes_body(int64_t n, int32_t r, const uint32_t* __restrict__ codes,
                                                          const double* __restrict__ mean,
                                                          const double* __restrict__ box_lo,
                                                          const double* __restrict__ box_hi,
                                                          const int* __restrict__ only_if,
                                                          double* __restrict__ x_new,
                                                          double* __restrict__ logw_new, int bx_, int gx_) {
#pragma clang fp contract(off)
  if (only_if && *only_if == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t gt = (int64_t)bx_ * blockDim.x + threadIdx.x;
  const int64_t wave = gt >> 6;
  const int64_t nwaves = ((int64_t)gx_ * blockDim.x) >> 6;
  // coordinate k of node i from its code (the same arithmetic as the Sobol mapping)
  auto node = [&](uint32_t code, double lo, double hi, double mk, double& xv, double& acc, int& b) {
    const double c = __dmul_rn(0.5, __dadd_rn(lo, hi));
    const double hw = __dmul_rn(0.5, __dsub_rn(hi, lo));
    const double u = __dsub_rn((double)code * 0x1p-31, 1.0);
    xv = __dadd_rn(c, __dmul_rn(hw, u));
    b |= (fabs(xv - lo) <= kBoundaryTol) || (fabs(hi - xv) <= kBoundaryTol);
    const double dv = __dsub_rn(xv, mk);
    acc = __dadd_rn(acc, __dmul_rn(dv, dv));
  };
  // 8- and 16-byte accesses to pairs of coordinates when the rows allow it
  const bool pairs = (r & 1) == 0 && ((reinterpret_cast<uintptr_t>(codes) & 7) |
                                      ((reinterpret_cast<uintptr_t>(x_new) | reinterpret_cast<uintptr_t>(box_lo) |
                                        reinterpret_cast<uintptr_t>(box_hi) | reinterpret_cast<uintptr_t>(mean)) &
                                       15)) == 0;
  // the box and the mean staged in LDS for rows of up to 2 kStagePairs coordinates (every
  // row reads them all; from LDS they leave the vector memory path to the codes and the nodes)
  constexpr int kStagePairs = 512;
  __shared__ double2 s_lo[kStagePairs], s_hi[kStagePairs], s_mk[kStagePairs];
  const double2* lo2 = reinterpret_cast<const double2*>(box_lo);
  const double2* hi2 = reinterpret_cast<const double2*>(box_hi);
  const double2* m2 = reinterpret_cast<const double2*>(mean);
  const bool staged = pairs && r <= 2 * kStagePairs;
  if (staged) {
    for (int p = threadIdx.x; p < r / 2; p += blockDim.x) {
      s_lo[p] = lo2[p];
      s_hi[p] = hi2[p];
      s_mk[p] = m2[p];
    }
    __syncthreads();
  }
  for (int64_t i = wave; i < n; i += nwaves) {
    double acc = 0.0;
    int b = 0;
    if (pairs) {
      const uint2* c2 = reinterpret_cast<const uint2*>(codes + (size_t)i * r);
      double2* x2 = reinterpret_cast<double2*>(x_new + (size_t)i * r);
      for (int32_t kk = lane; kk < r / 2; kk += 64) {
        const uint2 cd = c2[kk];
        const double2 lo = staged ? s_lo[kk] : lo2[kk], hi = staged ? s_hi[kk] : hi2[kk];
        const double2 mk = staged ? s_mk[kk] : m2[kk];
        double2 xv;
        node(cd.x, lo.x, hi.x, mk.x, xv.x, acc, b);
        node(cd.y, lo.y, hi.y, mk.y, xv.y, acc, b);
        x2[kk] = xv;
      }
    } else {
      for (int32_t k = lane; k < r; k += 64) {
        double xv;
        node(codes[(size_t)i * r + k], box_lo[k], box_hi[k], mean[k], xv, acc, b);
        x_new[(size_t)i * r + k] = xv;
      }
    }
    acc = wave_sum(acc);
    b = wave_or(b);
    if (lane == 0) logw_new[i] = b ? -INFINITY : -0.5 * acc;
  }
}

__global__ void __launch_bounds__(kBlock) k_restart_nodes(int64_t n, int32_t r, const uint32_t* __restrict__ codes,
                                                          const double* __restrict__ mean,
                                                          const double* __restrict__ box_lo,
                                                          const double* __restrict__ box_hi,
                                                          const int* __restrict__ only_if,
                                                          double* __restrict__ x_new,
                                                          double* __restrict__ logw_new) {
  k_restart_nodes_body(n, r, codes, mean, box_lo, box_hi, only_if, x_new, logw_new, blockIdx.x, gridDim.x);
}

// The resampling offsets (block 0, one block as k_rs_offsets) beside the new nodes in the
// plain box (the other blocks, as k_restart_nodes): the nodes read neither the weights nor
// the resampling buffers, so the two share a launch.
__global__ void __launch_bounds__(kBlock) k_rs_offsets_nodes(int nb, unsigned long long* __restrict__ tot, int64_t n,
                                                             int32_t r, const uint32_t* __restrict__ codes,
                                                             const double* __restrict__ mean,
                                                             const double* __restrict__ box_lo,
                                                             const double* __restrict__ box_hi,
                                                             double* __restrict__ x_new, double* __restrict__ logw_new,
                                                             int node_blocks) {
  if (blockIdx.x == 0) k_rs_offsets_body(nb, tot, 0, 1);
  else k_restart_nodes_body(n, r, codes, mean, box_lo, box_hi, nullptr, x_new, logw_new, blockIdx.x - 1, node_blocks);
}

__global__ void __launch_bounds__(kBlock) k_restart_nodes_batch(const restart_nodes_args* __restrict__ A,
                                                                const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const restart_nodes_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_restart_nodes_body(a.n, a.r, a.codes, a.mean, a.box_lo, a.box_hi, a.only_if, a.x_new, a.logw_new,
                       blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


__device__ __forceinline__ void k_ess_check_body(const double* __restrict__ ess, double ess_min,
                                                 uint32_t* __restrict__ flags, int bx_, int gx_) {
  if (threadIdx.x == 0 && bx_ == 0 && *ess < ess_min) atomicOr(flags, YY_FLAG_LOW_ESS);
}

__global__ void __launch_bounds__(kBlock) k_ess_check(const double* __restrict__ ess, double ess_min,
                                                      uint32_t* __restrict__ flags) {
  k_ess_check_body(ess, ess_min, flags, blockIdx.x, gridDim.x);
}

// The first resampling kernel of a single run with the restart's independent small
// steps folded in, to save their launches: the ESS check (block 0, where ess is
// given) and the plain restart box (where box_lo is given; the coordinates grid-
// strided over the blocks, the same arithmetic as k_box_plain).
__global__ void __launch_bounds__(kBlock) k_rs_local_front(int64_t n, const double* __restrict__ w,
                                                           unsigned long long* __restrict__ C,
                                                           unsigned long long* __restrict__ tot,
                                                           const double* __restrict__ ess, double ess_min,
                                                           uint32_t* __restrict__ flags, int32_t r, double R,
                                                           const double* __restrict__ mean,
                                                           double* __restrict__ box_lo, double* __restrict__ box_hi) {
  if (ess) k_ess_check_body(ess, ess_min, flags, blockIdx.x, gridDim.x);
  if (box_lo) {
    for (int64_t d = (int64_t)blockIdx.x * kBlock + threadIdx.x; d < r; d += (int64_t)gridDim.x * kBlock) {
      box_lo[d] = __dsub_rn(mean[d], R);
      box_hi[d] = __dadd_rn(mean[d], R);
    }
  }
  k_rs_local_body(n, w, C, tot, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_ess_check_batch(const ess_check_args* __restrict__ A,
                                                            const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const ess_check_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_ess_check_body(a.ess, a.ess_min, a.flags, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}



// Host launchers of the batched kernels (one block range per argument set).
yy_status launch_batched(hipStream_t st, const rs_local_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_rs_local_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_rs_local_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const rs_offsets_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_rs_offsets_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_rs_offsets_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const rs_add_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_rs_add_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_rs_add_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const rs_search_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_rs_search_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_rs_search_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const box_plain_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_box_plain_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_box_plain_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const restart_nodes_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_restart_nodes_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_restart_nodes_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const ess_check_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_ess_check_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_ess_check_batch");
  return YY_OK;
}

}  // namespace yy

using namespace yy;

__global__ void k_set_int(int32_t* p, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

extern "C" yy_status yy_restart(yy_ctx ctx, int64_t n, int32_t r, const uint32_t* codes, const double* x_cur,
                                const double* w, const double* mean, const double* ess, int64_t step,
                                const yy_restart_params* params, int64_t* idx, double* box_lo,
                                double* box_hi, double* x_new, double* logw_new, int32_t* used) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_restart: ctx is NULL");
  if (!params) return fail(YY_ERR_ARG, "yy_restart: params is NULL");
  if (n < 1 || n > ((int64_t)1 << 32)) return fail(YY_ERR_ARG, "yy_restart: n out of range");
  if (r < 1 || r > YY_MAX_R) return fail(YY_ERR_ARG, "yy_restart: r out of range");
  if (!(params->R > 0.0) || !std::isfinite(params->R)) return fail(YY_ERR_ARG, "yy_restart: R must be positive");
  if (!codes || !mean || !box_lo || !box_hi || !x_new || !logw_new)
    return fail(YY_ERR_ARG, "yy_restart: NULL array");
  if (idx && !w) return fail(YY_ERR_ARG, "yy_restart: resampling needs w");
  yy_proposal prop = params->proposal;
  if (prop) {
    if (!x_cur || !idx) return fail(YY_ERR_ARG, "yy_restart: a learned proposal needs x_cur and idx");
    if (x_cur == x_new) return fail(YY_ERR_ARG, "yy_restart: x_cur must not alias x_new");
    if (prop->ctx != ctx || prop->r != r) return fail(YY_ERR_ARG, "yy_restart: proposal of another context or r");
    if (!(params->cover_min >= 0.0 && params->cover_min <= 1.0))
      return fail(YY_ERR_ARG, "yy_restart: cover_min must be in [0, 1]");
  }
  YY_HIP(hipSetDevice(ctx->device));
  // with resampling, the ESS check and the plain box run inside its first kernel
  const bool front = idx != nullptr;
  if (ess && !front) {
    k_ess_check<<<1, 64, 0, ctx->stream>>>(ess, params->ess_min, ctx->d_flags);
    YY_LAUNCH_CHECK("k_ess_check");
  }
  int64_t blocks = (n + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  if (blocks * kBlock < r) blocks = (r + kBlock - 1) / kBlock;
  // plain box with resampling: the new nodes go out beside the resampling offsets, unless the caller's
  // arrays overlap so that the order between them matters
  auto overlaps = [](const void* a, size_t na, const void* b, size_t nb_) {
    const char *pa = static_cast<const char*>(a), *pb = static_cast<const char*>(b);
    return pa && pb && pa < pb + nb_ && pb < pa + na;
  };
  const size_t xb = (size_t)n * r * sizeof(double), nbytes = (size_t)n * sizeof(double);
  const bool early_nodes =
      front && !prop && !overlaps(w, nbytes, x_new, xb) && !overlaps(w, nbytes, logw_new, nbytes) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), x_new, xb) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), logw_new, nbytes) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), mean, (size_t)r * sizeof(double)) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), box_lo, (size_t)r * sizeof(double)) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), box_hi, (size_t)r * sizeof(double)) &&
      !overlaps(idx, (size_t)n * sizeof(int64_t), codes, (size_t)n * r * sizeof(uint32_t));
  if (idx) {
    const int nb = (int)((n + kBlock - 1) / kBlock);
    yy_status st = ctx->scan.ensure(((size_t)n + nb + 1) * sizeof(unsigned long long));
    if (st != YY_OK) return st;
    unsigned long long* C = ctx->scan.as<unsigned long long>();
    unsigned long long* tot = C + n;
    k_rs_local_front<<<nb, kBlock, 0, ctx->stream>>>(n, w, C, tot, ess, params->ess_min, ctx->d_flags, r,
                                                     params->R, mean, prop ? nullptr : box_lo,
                                                     prop ? nullptr : box_hi);
    YY_LAUNCH_CHECK("k_rs_local_front");
    if (early_nodes) {
      k_rs_offsets_nodes<<<(unsigned)blocks + 1, kBlock, 0, ctx->stream>>>(nb, tot, n, r, codes, mean, box_lo, box_hi,
                                                                           x_new, logw_new, (int)blocks);
      YY_LAUNCH_CHECK("k_rs_offsets_nodes");
    } else {
      k_rs_offsets<<<1, kBlock, 0, ctx->stream>>>(nb, tot);
      YY_LAUNCH_CHECK("k_rs_offsets");
    }
    k_rs_add<<<nb, kBlock, 0, ctx->stream>>>(n, tot, C);
    YY_LAUNCH_CHECK("k_rs_add");
    const uint64_t U = h_sm64(h_sm64(params->seed, kDomainResample), (uint64_t)step) >> 32;
    k_rs_search<<<nb, kBlock, 0, ctx->stream>>>(n, nb, tot, C, U, idx, ctx->d_flags);
    YY_LAUNCH_CHECK("k_rs_search");
  }
  int* dec = nullptr;
  if (prop) {
    yy_status st = proposal_restart_prepare(ctx, prop, n, r, x_cur, idx, mean, params->R, params->cover_min,
                                            box_lo, box_hi, &dec);
    if (st != YY_OK) return st;
  } else if (!front) {
    k_box_plain<<<(unsigned)((r + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(r, params->R, mean, box_lo,
                                                                                 box_hi);
    YY_LAUNCH_CHECK("k_box_plain");
  }
  if (!early_nodes) {
    k_restart_nodes<<<(unsigned)blocks, kBlock, 0, ctx->stream>>>(n, r, codes, mean, box_lo, box_hi, nullptr,
                                                                  x_new, logw_new);
    YY_LAUNCH_CHECK("k_restart_nodes");
  }
  if (prop) {
    yy_status st = proposal_restart_finish(ctx, prop, n, r, logw_new, mean, params->R, params->ess_min, box_lo,
                                           box_hi, dec, used);
    if (st != YY_OK) return st;
    k_restart_nodes<<<(unsigned)blocks, kBlock, 0, ctx->stream>>>(n, r, codes, mean, box_lo, box_hi, dec + 1,
                                                                  x_new, logw_new);
    YY_LAUNCH_CHECK("k_restart_nodes");
  } else if (used) {
    k_set_int<<<1, 64, 0, ctx->stream>>>(used, 0);
    YY_LAUNCH_CHECK("k_set_int");
  }
  return YY_OK;
}
