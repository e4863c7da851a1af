// yy_propagate.hip -- the prediction step (Sec. 4 kernel operator in push form,
// Sec. 4.3.3 multi-scale combination, Sec. 9 log-domain prediction).
//
//   logw_out[i] = log( sum_s c_s dV sum_j N(x_i; x_j + tau_s f(x_j), q tau_s I) e^{logw_in[j]}
//                      + c_S e^{logw_in[i]} )
//
// Stages: (1) prepare the node set once per node version: centred FP32
// coordinates, f(x), BF16 hi/lo splits, per-node norms, boundary flags, the box
// volume and the norm maxima used by the near-pair error bound; (2) source
// weights relative to their maximum in base 2; (3) pairwise kernel: for every
// target i and scale s a running (max, sum) over sources in base 2; (4) FP64
// combination of the scales with the Gaussian constants, the quadrature
// weight and the identity term.
#include <algorithm>
#include <climits>
#include <cmath>

#include <vector>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

// ---------------------------------------------------------------------------
// (1) node preparation: W lanes per node -- W = 16, one wavefront per 4
// consecutive nodes, or where n_pad <= kPrepWideMax W = 64, a wavefront per
// node, so that a small node set's rows are walked in fewer dependent steps.
// Rows of even length take two 2W-wide K ranges per step, a coordinate pair per
// lane in each (with W = 16 whole 128-byte lines of the row-major planes, and
// of the tiled planes: 4 nodes x 16 K values per chunk); other rows one W-wide
// K range per step, a coordinate per lane.  Single runs and the batched step
// choose W by the same rule, so their node norms agree bit for bit.
// Matrix-core planes are tiled [plane][rp/16][n_pad][16] so that 16 K values
// of consecutive nodes are contiguous; rows n..n_pad-1 are zero.
template <int W>
__device__ inline double sum_node(double v) {   // over the W lanes of a node
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// MODE 0 writes everything; MODE 1 (BF16X3P, deferred planes) the node norms, the
// boundary flags, the maxima and hi(xc) over the first kPreK coordinates; MODE 2
// the planes and rows only (the rest of a MODE 1 preparation).
template <int MODE, int W>
__device__ __forceinline__ void k_prepare_body(int64_t n, int64_t n_pad, int32_t r, int32_t rp,
                                                    int32_t drift, const double* __restrict__ A,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ lo,
                                                    const double* __restrict__ hi,
                                                    float* __restrict__ xc32, float* __restrict__ f32,
                                                    uint16_t* __restrict__ bf, float* __restrict__ f32t,
                                                    double* __restrict__ node, int* __restrict__ bnd,
                                                    int bx_, int gx_, const double* __restrict__ fgiven = nullptr,
                                                    const int* __restrict__ bnd_given = nullptr) {
  // fgiven: drift values [n][r] when drift == kDriftGiven (a whitened node set); bnd_given: the
  // boundary flags, when the box test does not apply to these coordinates
  static_assert(W == 16 || W == 64, "16 or 64 lanes per node");
  constexpr int NPW = 64 / W;   // nodes per wave
  const int lane = threadIdx.x & 63, sub = lane / W, kl = lane % W;
  const int64_t wave = ((int64_t)bx_ * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gx_ * blockDim.x) >> 6;
  const size_t plane = (size_t)n_pad * rp;
  static_assert(kPreK % 32 == 0, "the prefix is whole coordinate pairs");
  double mx[4] = {0.0, 0.0, 0.0, 0.0};   // running maxima of the norms (all >= 0)
  // Rows of even length with 16-byte aligned x, lo and hi take the paired path: each lane handles
  // the coordinate pairs k0 + 2 kl and k0 + 2 W + 2 kl (16-byte loads, 8-byte stores), 4 W
  // coordinates per step; the linear drift keeps one coordinate per lane.  A lane's prefix sums
  // (the first kPreK coordinates) are its running sums after its last coordinate below kPreK.
  const bool pairs = (r & 1) == 0 && drift != YY_F_LINEAR &&
                     ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(lo) |
                       reinterpret_cast<uintptr_t>(hi) | reinterpret_cast<uintptr_t>(fgiven)) & 15) == 0;
  auto near_box = [](double xv, double l, double h) {
    return (int)((fabs(xv - l) <= kBoundaryTol) || (fabs(h - xv) <= kBoundaryTol));
  };
  auto sinmix = [](double xv, double xn) {
    return sin(xv) * (-0.5 * xv + 0.1 * xn) + sin(2.0 * xv) * (-0.3 * xv + 0.3 * xn);
  };
  // BF16 hi part of v (the FP32 value of d) and the BF16 of what it leaves of d
  auto split = [](double d, float v, uint32_t& h, uint32_t& l) {
    const uint16_t hv = f32_to_bf16(v);
    h = hv;
    l = f32_to_bf16((float)(d - (double)bf16_to_f32(hv)));
  };
  for (int64_t i4 = wave * NPW; i4 < n_pad; i4 += nwaves * NPW) {
    const int64_t i = i4 + sub;   // n_pad is a multiple of 4
    const bool real = i < n;
    const double* xi = x + (size_t)(real ? i : 0) * r;
    double sxx = 0.0, sff = 0.0, sxf = 0.0;
    double pxx = 0.0, pff = 0.0, pxf = 0.0;   // over the first kPreK coordinates
    int b = 0;
    if (pairs) {
      for (int32_t k0 = 0; k0 < rp; k0 += 4 * W) {
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
          const int32_t k = k0 + 2 * W * half + 2 * kl;
          double xc0 = 0.0, xc1 = 0.0, f0 = 0.0, f1 = 0.0;
          if (real && k < r) {   // r is even: both coordinates of the pair are inside
            const double2 xv = *reinterpret_cast<const double2*>(xi + k);
            const double2 l2 = *reinterpret_cast<const double2*>(lo + k);
            const double2 h2 = *reinterpret_cast<const double2*>(hi + k);
            xc0 = xv.x - 0.5 * (l2.x + h2.x);
            xc1 = xv.y - 0.5 * (l2.y + h2.y);
            if (!bnd_given) b |= near_box(xv.x, l2.x, h2.x) | near_box(xv.y, l2.y, h2.y);
            if (drift == YY_F_COS) {
              f0 = cos(xv.x);
              f1 = cos(xv.y);
            } else if (drift == YY_F_PAPER_SINMIX) {
              f0 = sinmix(xv.x, xv.y);
              f1 = sinmix(xv.y, k + 2 < r ? xi[k + 2] : 0.0);
            } else if (drift == kDriftGiven) {
              const double2 fv = *reinterpret_cast<const double2*>(fgiven + (size_t)i * r + k);
              f0 = fv.x;
              f1 = fv.y;
            }
            sxx = fma(xc0, xc0, sxx);
            sff = fma(f0, f0, sff);
            sxf = fma(xc0, f0, sxf);
            sxx = fma(xc1, xc1, sxx);
            sff = fma(f1, f1, sff);
            sxf = fma(xc1, f1, sxf);
          }
          if (k < kPreK) {
            pxx = sxx;
            pff = sff;
            pxf = sxf;
          }
          // rp is a multiple of 32: the pair is inside or outside as a whole
          if (k < (MODE == 1 ? min(rp, kPreK) : rp)) {
            const float a0 = (float)xc0, a1 = (float)xc1, g0 = (float)f0, g1 = (float)f1;
            if (MODE == 1) {
              uint32_t xh0, xl0, xh1, xl1;
              split(xc0, a0, xh0, xl0);
              split(xc1, a1, xh1, xl1);
              *reinterpret_cast<uint32_t*>(bf + ((size_t)(k >> 4) * n_pad + i) * 16 + (k & 15)) = xh0 | (xh1 << 16);
              continue;
            }
            if (real) {
              const size_t o = (size_t)i * rp + k;
              *reinterpret_cast<float2*>(xc32 + o) = make_float2(a0, a1);
              *reinterpret_cast<float2*>(f32 + o) = make_float2(g0, g1);
            }
            const size_t t = ((size_t)(k >> 4) * n_pad + i) * 16 + (k & 15);
            if (bf) {
              uint32_t xh0, xl0, xh1, xl1, fh0, fl0, fh1, fl1;
              split(xc0, a0, xh0, xl0);
              split(xc1, a1, xh1, xl1);
              split(f0, g0, fh0, fl0);
              split(f1, g1, fh1, fl1);
              *reinterpret_cast<uint32_t*>(bf + t) = xh0 | (xh1 << 16);
              *reinterpret_cast<uint32_t*>(bf + plane + t) = fh0 | (fh1 << 16);
              *reinterpret_cast<uint32_t*>(bf + 2 * plane + t) = xl0 | (xl1 << 16);
              *reinterpret_cast<uint32_t*>(bf + 3 * plane + t) = fl0 | (fl1 << 16);
            }
            if (f32t) {
              *reinterpret_cast<float2*>(f32t + t) = make_float2(a0, a1);
              *reinterpret_cast<float2*>(f32t + plane + t) = make_float2(g0, g1);
            }
          }
        }
      }
    } else {
      for (int32_t k0 = 0; k0 < rp; k0 += W) {
        const int32_t k = k0 + kl;
        float xcv = 0.f, fv = 0.f;
        double xcd = 0.0, fd = 0.0;
        if (real && k < r) {
          const double xv = xi[k];
          const double c = 0.5 * (lo[k] + hi[k]);
          xcd = xv - c;
          if (!bnd_given) b |= near_box(xv, lo[k], hi[k]);
          if (drift == YY_F_COS) {
            fd = cos(xv);
          } else if (drift == kDriftGiven) {
            fd = fgiven[(size_t)i * r + k];
          } else if (drift == YY_F_LINEAR) {
            const double* Ak = A + (size_t)k * r;
            double acc = 0.0;
            for (int32_t l = 0; l < r; ++l) acc = fma(Ak[l], xi[l], acc);
            fd = acc;
          } else if (drift == YY_F_PAPER_SINMIX) {
            fd = sinmix(xv, k + 1 < r ? xi[k + 1] : 0.0);
          }
          sxx = fma(xcd, xcd, sxx);
          sff = fma(fd, fd, sff);
          sxf = fma(xcd, fd, sxf);
          xcv = (float)xcd;
          fv = (float)fd;
        }
        if (k < kPreK) {
          pxx = sxx;
          pff = sff;
          pxf = sxf;
        }
        if (k >= rp) continue;   // (W = 64 runs past r_p where r_p = 32: no plane or row holds those)
        const size_t t = ((size_t)(k >> 4) * n_pad + i) * 16 + (k & 15);
        if (MODE == 1) {
          if (k < kPreK) bf[t] = f32_to_bf16(xcv);
          continue;
        }
        if (real) {
          const size_t o = (size_t)i * rp + k;
          xc32[o] = xcv;
          f32[o] = fv;
        }
        if (bf) {
          const uint16_t xh = f32_to_bf16(xcv);
          const uint16_t xl = f32_to_bf16((float)(xcd - (double)bf16_to_f32(xh)));
          const uint16_t fh = f32_to_bf16(fv);
          const uint16_t fl = f32_to_bf16((float)(fd - (double)bf16_to_f32(fh)));
          bf[t] = xh;
          bf[plane + t] = fh;
          bf[2 * plane + t] = xl;
          bf[3 * plane + t] = fl;
        }
        if (f32t) {
          f32t[t] = xcv;
          f32t[plane + t] = fv;
        }
      }
    }
    if (MODE == 2) continue;
    sxx = sum_node<W>(sxx);
    sff = sum_node<W>(sff);
    sxf = sum_node<W>(sxf);
    pxx = sum_node<W>(pxx);
    pff = sum_node<W>(pff);
    pxf = sum_node<W>(pxf);
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) b |= __shfl_xor(b, off, 64);
    if (bnd_given && real) b = bnd_given[i];
    if (kl == 0 && real) {
      node[i] = sxx;
      node[n + i] = sff;
      node[2 * n + i] = sxf;
      node[3 * n + i] = pxx;
      node[4 * n + i] = pff;
      node[5 * n + i] = pxf;
      bnd[i] = b;
    }
    if (real) {
      mx[0] = fmax(mx[0], sxx);
      mx[1] = fmax(mx[1], sff);
      mx[2] = fmax(mx[2], pxx);
      mx[3] = fmax(mx[3], pff);
    }
  }
  if (MODE == 2) return;
  // the block's maxima of |xc|^2, |f|^2 and their first-kPreK parts, to
  // node[6 n + 4 bx + c] (k_prepare_scalars reduces them)
  __shared__ double sh[kBlock / 64];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double v = block_max<kBlock>(mx[c], sh);
    if (threadIdx.x == 0) node[6 * n + 4 * (int64_t)bx_ + c] = v;
  }
}

int prepare_blocks(int64_t n_pad) {
  return prep_wide(n_pad) ? (int)(n_pad / 4) : (int)std::min<int64_t>((n_pad + 15) / 16, 16384);
}

// MODE 1 marks the deferred planes as not yet written (defer[1] = 0).
template <int MODE>
__global__ void __launch_bounds__(kBlock, 4) k_prepare(int64_t n, int64_t n_pad, int32_t r, int32_t rp,
                                                       int32_t drift, const double* __restrict__ A,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ lo,
                                                       const double* __restrict__ hi,
                                                       float* __restrict__ xc32, float* __restrict__ f32,
                                                       uint16_t* __restrict__ bf, float* __restrict__ f32t,
                                                       double* __restrict__ node, int* __restrict__ bnd,
                                                       int* __restrict__ defer, const double* __restrict__ fgiven,
                                                       const int* __restrict__ bnd_given) {
  if (MODE == 1 && blockIdx.x == 0 && threadIdx.x == 0) defer[1] = 0;
  if (prep_wide(n_pad))
    k_prepare_body<MODE, 64>(n, n_pad, r, rp, drift, A, x, lo, hi, xc32, f32, bf, f32t, node, bnd, blockIdx.x,
                             gridDim.x, fgiven, bnd_given);
  else
    k_prepare_body<MODE, 16>(n, n_pad, r, rp, drift, A, x, lo, hi, xc32, f32, bf, f32t, node, bnd, blockIdx.x,
                             gridDim.x, fgiven, bnd_given);
}

// The rest of a MODE 1 preparation, after the screen: every block returns at
// once unless the screen flagged a tile in this call and the planes are not
// yet complete (k_combine then marks them complete).
__global__ void __launch_bounds__(kBlock, 4) k_prepare_rest(DeferredPrep d) {
  if (d.defer[0] == 0 || d.defer[1] != 0) return;
  if (prep_wide(d.n_pad))
    k_prepare_body<2, 64>(d.n, d.n_pad, d.r, d.rp, d.drift, d.A, d.x, d.lo, d.hi, d.xc32, d.f32, d.bf, nullptr,
                          nullptr, nullptr, blockIdx.x, gridDim.x);
  else
    k_prepare_body<2, 16>(d.n, d.n_pad, d.r, d.rp, d.drift, d.A, d.x, d.lo, d.hi, d.xc32, d.f32, d.bf, nullptr,
                          nullptr, nullptr, blockIdx.x, gridDim.x);
}

yy_status launch_prepare_rest(hipStream_t st, const DeferredPrep& d) {
  k_prepare_rest<<<(unsigned)prepare_blocks(d.n_pad), kBlock, 0, st>>>(d);
  YY_LAUNCH_CHECK("k_prepare_rest");
  return YY_OK;
}

__global__ void __launch_bounds__(kBlock, 4) k_prepare_batch(const prepare_args* __restrict__ A,
                                                          const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const prepare_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  if (prep_wide(a.n_pad))
    k_prepare_body<0, 64>(a.n, a.n_pad, a.r, a.rp, a.drift, a.A, a.x, a.lo, a.hi, a.xc32, a.f32, a.bf, a.f32t, a.node,
                          a.bnd, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
  else
    k_prepare_body<0, 16>(a.n, a.n_pad, a.r, a.rp, a.drift, a.A, a.x, a.lo, a.hi, a.xc32, a.f32, a.bf, a.f32t, a.node,
                          a.bnd, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// Box volume (log) and the maxima of |xc| and |f| (all coordinates and the
// first kPreK) from the nparts per-block maxima of k_prepare: one block.
__device__ __forceinline__ void k_prepare_scalars_body(int64_t n, int32_t r, int32_t nparts,
                                                            const double* __restrict__ lo,
                                                            const double* __restrict__ hi,
                                                            const double* __restrict__ node,
                                                            double* __restrict__ scal, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  double lv = 0.0;
  for (int32_t k = threadIdx.x; k < r; k += kBlock) lv += log(hi[k] - lo[k]);
  lv = block_sum<kBlock>(lv, sh);
  const double* part = node + 6 * n;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t p = threadIdx.x; p < nparts; p += kBlock)
#pragma unroll
    for (int c = 0; c < 4; ++c) m[c] = fmax(m[c], part[4 * (int64_t)p + c]);
#pragma unroll
  for (int c = 0; c < 4; ++c) m[c] = block_max<kBlock>(m[c], sh);
  if (threadIdx.x == 0) {
    scal[0] = lv;
    scal[1] = sqrt(m[0]);
    scal[2] = sqrt(m[1]);
    scal[3] = 0.0;
    scal[4] = sqrt(m[2]);
    scal[5] = sqrt(m[3]);
  }
}

__global__ void __launch_bounds__(kBlock) k_prepare_scalars(int64_t n, int32_t r, int32_t nparts,
                                                            const double* __restrict__ lo,
                                                            const double* __restrict__ hi,
                                                            const double* __restrict__ node,
                                                            double* __restrict__ scal) {
  k_prepare_scalars_body(n, r, nparts, lo, hi, node, scal, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_prepare_scalars_batch(const prepare_scalars_args* __restrict__ A,
                                                                  const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const prepare_scalars_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_prepare_scalars_body(a.n, a.r, a.nparts, a.lo, a.hi, a.node, a.scal, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// ---------------------------------------------------------------------------
// (2) source weights: lw2[j] = (logw[j] - max_valid logw) * log2(e), -inf for
// boundary nodes and zero weights.  Two kernels: block maxima, then every
// block re-reduces the (short) list of block maxima in the same order.
__device__ __forceinline__ void k_lw_max_body(int64_t n, const double* __restrict__ lw,
                                                   const int* __restrict__ bnd,
                                                   double* __restrict__ part, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  double m = -INFINITY;
  for (int64_t j = (int64_t)bx_ * kBlock + threadIdx.x; j < n; j += (int64_t)gx_ * kBlock)
    if (!bnd[j]) m = fmax(m, lw[j]);
  m = block_max<kBlock>(m, sh);
  if (threadIdx.x == 0) part[bx_] = m;
}

__global__ void __launch_bounds__(kBlock) k_lw_max(int64_t n, const double* __restrict__ lw,
                                                   const int* __restrict__ bnd,
                                                   double* __restrict__ part) {
  k_lw_max_body(n, lw, bnd, part, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_lw_max_batch(const lw_max_args* __restrict__ A,
                                                         const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const lw_max_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_lw_max_body(a.n, a.lw, a.bnd, a.part, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


__device__ __forceinline__ void k_lw_convert_body(int64_t n, int nparts,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ lw,
                                                       const int* __restrict__ bnd,
                                                       float* __restrict__ lw2,
                                                       double* __restrict__ ref_out, int bx_, int gx_,
                                                       long long* __restrict__ heavy = nullptr) {
  __shared__ double sh[kBlock / 64];
  double m = -INFINITY;
  for (int p = threadIdx.x; p < nparts; p += kBlock) m = fmax(m, part[p]);
  m = block_max<kBlock>(m, sh);
  if (bx_ == 0 && threadIdx.x == 0) *ref_out = m;
  long long cand = LLONG_MAX;   // this thread's first valid source attaining the maximum
  for (int64_t j = (int64_t)bx_ * kBlock + threadIdx.x; j < n; j += (int64_t)gx_ * kBlock) {
    const double v = lw[j];
    const bool valid = !bnd[j] && v != -INFINITY && m != -INFINITY;
    lw2[j] = valid ? (float)((v - m) * kLog2e) : -INFINITY;
    if (valid && v == m && cand == LLONG_MAX) cand = j;
  }
  if (heavy) {
    // per block: the smallest such index (heavy[bx], LLONG_MAX for none); k_heavy reduces them
    __shared__ long long sj;
    if (threadIdx.x == 0) sj = LLONG_MAX;
    __syncthreads();
    if (cand != LLONG_MAX) atomicMin(&sj, cand);
    __syncthreads();
    if (threadIdx.x == 0) heavy[bx_] = sj;
  }
}

__global__ void __launch_bounds__(kBlock) k_lw_convert(int64_t n, int nparts,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ lw,
                                                       const int* __restrict__ bnd,
                                                       float* __restrict__ lw2,
                                                       double* __restrict__ ref_out,
                                                       long long* __restrict__ heavy) {
  k_lw_convert_body(n, nparts, part, lw, bnd, lw2, ref_out, blockIdx.x, gridDim.x, heavy);
}

// ---------------------------------------------------------------------------
// Lower bound of every (scale, target) row maximum for the matrix-core forms
// (push form): the larger of the exact self-pair exponent and the exact
// exponent of the pair with the heaviest source j* (a term of the row, in FP64
// direct differences: lw2_j* = 0, d = x_i - x_j* - tau_s f(x_j*)).  The second
// is formed only for rows whose self term lies more than kRowRefGap bits below
// the heaviest weight; elsewhere the self term is within kRowRefGap bits of
// any term the heaviest source could give.  Where it is formed, that exact
// term is also kept (rhv): the pairwise kernels count the pair (i, j*) at
// initialisation from it, as they count the self pair, and leave it out of
// their tiles and screens, so a posterior collapsed onto one node flags no
// tile for its sake.  Rows: x (the nodes, or with
// general noise their whitened images; the box centre cancels in the
// differences).  k_heavy (one block) reduces the conversion blocks' candidates
// to j* (the first valid source of maximal weight) and evaluates f(x_j*) once;
// k_row_ref takes a wave per target with the lanes across the coordinates (4 or
// 16 targets per block, row_ref_targets), or where r <= 256 16 targets of 16
// lanes each.
constexpr float kRowRefGap = 160.f;
constexpr int kRowRefTargets = 16;

__device__ __forceinline__ void k_row_ref_body(const RowRefArgs& a, int bx_) {
  __shared__ float sself[YY_MAX_SCALES][kRowRefTargets];
  __shared__ int sneed[kRowRefTargets];
  const int T = row_ref_targets(a.r, a.n);   // <= kRowRefTargets
  const int64_t i0 = (int64_t)bx_ * T;
  const long long js = *a.jstar;
  if (threadIdx.x < T) {
    const int64_t i = i0 + threadIdx.x;
    bool need = false;
    if (i < a.n) {
      const float li = a.lw2[i];
      const double nf = a.node[a.n + i];
      for (int s = 0; s < a.S; ++s) {
        const float self = (li != -INFINITY && !a.bnd[i]) ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf)
                                                          : -INFINITY;
        sself[s][threadIdx.x] = self;
        need |= self < -kRowRefGap;
      }
      need = need && js >= 0 && js != i && !a.bnd[i];
    }
    sneed[threadIdx.x] = need;
  }
  __syncthreads();
  // lanes per target: the whole wave across the coordinates of a long row; for r <= 256, groups of 16
  // lanes, four targets per wave at a time (the shuffles stay inside a group and run in converged flow)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int L = a.r > 256 ? 64 : 16;
  const int per = 64 / L, sg = lane / L, sl = lane % L;
  for (int u0 = wave * per; u0 < T; u0 += (kBlock / 64) * per) {
    const int u = u0 + sg;   // < T: u0 is a multiple of per, which divides T
    const int64_t i = i0 + u;
    const bool valid = i < a.n;
    const bool need = valid && sneed[u];
    // (scale loops unrolled to YY_MAX_SCALES so that D stays in registers)
    double D[YY_MAX_SCALES] = {0, 0, 0, 0, 0, 0};
    if (need) {
      const double* xi = a.x + (size_t)i * a.r;
      const double* xj = a.x + (size_t)js * a.r;
      for (int32_t k = sl; k < a.r; k += L) {
        const double d = xi[k] - xj[k], fk = a.fstar[k];
#pragma unroll
        for (int s = 0; s < YY_MAX_SCALES; ++s)
          if (s < a.S) {
            const double e = d - a.taud[s] * fk;
            D[s] = fma(e, e, D[s]);
          }
      }
    }
    if (__any(need))   // wave-uniform, so the shuffles run in converged flow; skipped where no row needs them
#pragma unroll
      for (int s = 0; s < YY_MAX_SCALES; ++s)
        if (s < a.S)
          for (int off = L / 2; off > 0; off >>= 1) D[s] += __shfl_xor(D[s], off, 64);
    if (valid && sl == 0)
#pragma unroll
      for (int s = 0; s < YY_MAX_SCALES; ++s) {
        if (s >= a.S) break;
        float ref = sself[s][u], hv = -INFINITY;
        if (need) {
          hv = (float)(-a.kapd[s] * D[s]);
          ref = fmaxf(ref, hv);
        }
        a.rref[(size_t)s * a.n + i] = ref;
        a.rhv[(size_t)s * a.n + i] = hv;
      }
  }
}

__global__ void __launch_bounds__(kBlock) k_row_ref(RowRefArgs a) { k_row_ref_body(a, blockIdx.x); }

// batched: the first block of each run's range evaluates its heavy source, the rows follow in a second launch
__global__ void __launch_bounds__(kBlock) k_heavy_batch(const RowRefArgs* __restrict__ A, const int* __restrict__ pre,
                                                        int nr) {
  if (!A[blockIdx.x].rref) return;   // a run in the vector-ALU form has no row floor
  k_heavy_body(A[blockIdx.x]);
}

__global__ void __launch_bounds__(kBlock) k_row_ref_batch(const RowRefArgs* __restrict__ A, const int* __restrict__ pre,
                                                          int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  k_row_ref_body(A[q], blockIdx.x - pre[q]);
}

__global__ void __launch_bounds__(kBlock) k_lw_convert_batch(const lw_convert_args* __restrict__ A,
                                                             const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const lw_convert_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_lw_convert_body(a.n, a.nparts, a.part, a.lw, a.bnd, a.lw2, a.ref_out, blockIdx.x - pre[q], pre[q + 1] - pre[q],
                    a.heavy);
}


// ---------------------------------------------------------------------------
// (3a) pairwise kernel on the vector ALUs (plain FP32 direct differences).
// Block: 64 targets x 64 sources, 256 threads, each thread 4 targets x 4
// sources x S scales.  The source range of one block is [j_begin, j_end).
// Each thread keeps its own running (max, sum) per (target, scale) across all
// its source tiles; the 16 threads that share targets merge at the end.
constexpr int kVI = 64, kVJ = 64;

// Push form: |x_i - x_j - tau f_j|^2; pull form: |x_i - tau f_i - x_j|^2 (the
// f rows of the targets instead of the sources).
// bx: the block of 64 targets, by: the source split (the batched launch takes both from its work item).
template <int S, int KC, bool PULL>
__device__ __forceinline__ void pair_valu_body(const PairArgs& a, int64_t j_per_split, const double* taud,
                                               const double* kapd, int bx, int by) {
  __shared__ float sxi[KC][kVI + 4];
  __shared__ float sxj[KC][kVJ + 4];
  __shared__ float sfj[KC][kVJ + 4];
  __shared__ float slw[kVJ];
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  const int64_t n = a.n;
  const int64_t i0 = (int64_t)bx * kVI;
  const int64_t jb = (int64_t)by * j_per_split;
  const int64_t je = jb + j_per_split < n ? jb + j_per_split : n;

  float M[4][S], Ssum[4][S];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      M[p][s] = -INFINITY;
      Ssum[p][s] = 0.f;
    }
  float tau[S], kap[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    tau[s] = a.tau[s];
    kap[s] = a.kap2[s];
  }

  for (int64_t j0 = jb; j0 < je; j0 += kVJ) {
    float acc[4][4][S];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < S; ++s) acc[p][q][s] = 0.f;
    __syncthreads();
    if (tid < kVJ) slw[tid] = (j0 + tid < je) ? a.lw2[j0 + tid] : -INFINITY;
    for (int k0 = 0; k0 < a.r; k0 += KC) {
      __syncthreads();
      // load KC dims of 64 targets and 64 sources (zero outside the ranges)
      for (int e = tid; e < 64 * KC; e += 256) {
        const int row = e / KC, kk = e % KC;
        const int k = k0 + kk;
        const int64_t gi = i0 + row, gj = j0 + row;
        const bool vi = (gi < n && k < a.r);
        sxi[kk][row] = vi ? a.xc[(size_t)gi * a.rp + k] : 0.f;
        const bool vj = (gj < je && k < a.r);
        sxj[kk][row] = vj ? a.xc[(size_t)gj * a.rp + k] : 0.f;
        if (PULL) sfj[kk][row] = vi ? a.f[(size_t)gi * a.rp + k] : 0.f;   // the targets' f rows
        else sfj[kk][row] = vj ? a.f[(size_t)gj * a.rp + k] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const float4 xi = *reinterpret_cast<const float4*>(&sxi[kk][ti * 4]);
        const float4 xj = *reinterpret_cast<const float4*>(&sxj[kk][tj * 4]);
        const float4 fj = *reinterpret_cast<const float4*>(&sfj[kk][(PULL ? ti : tj) * 4]);
        const float xia[4] = {xi.x, xi.y, xi.z, xi.w};
        const float xja[4] = {xj.x, xj.y, xj.z, xj.w};
        const float fja[4] = {fj.x, fj.y, fj.z, fj.w};
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float d = xia[p] - xja[q];
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const float e = fmaf(-tau[s], fja[PULL ? p : q], d);
              acc[p][q][s] = fmaf(e, e, acc[p][q][s]);
            }
          }
      }
    }
    // exponents and the running (max, sum)
    const bool diag = (j0 < i0 + kVI) && (i0 < j0 + kVJ);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int64_t gi = i0 + ti * 4 + p;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        float ev[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t gj = j0 + tj * 4 + q;
          float e = slw[tj * 4 + q] - kap[s] * acc[p][q][s];
          if (diag && gj == gi && gi < n) {
            // self pair: |tau_s f(x_i)|^2 from the FP64 norm
            e = slw[tj * 4 + q] - (float)(kapd[s] * taud[s] * taud[s] * a.node[n + gi]);
          }
          ev[q] = e;
        }
        const float m = fmaxf(fmaxf(ev[0], ev[1]), fmaxf(ev[2], ev[3]));
        if (m == -INFINITY) continue;
        if (m > M[p][s]) {
          Ssum[p][s] *= exp2f(M[p][s] - m);
          M[p][s] = m;
        }
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) t += exp2f(ev[q] - M[p][s]);
        Ssum[p][s] += t;
      }
    }
  }
  // merge the 16 threads (consecutive lanes) that share the same targets
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float m = M[p][s], sm = Ssum[p][s];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const float mo = __shfl_xor(m, off, 64);
        const float so = __shfl_xor(sm, off, 64);
        lse2_merge(m, sm, mo, so);
      }
      M[p][s] = m;
      Ssum[p][s] = sm;
    }
  if (tj == 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int64_t gi = i0 + ti * 4 + p;
      if (gi >= n) continue;
#pragma unroll
      for (int s = 0; s < S; ++s)
        a.part[((size_t)by * S + s) * n + gi] = make_float2(M[p][s], Ssum[p][s]);
    }
  }
}

template <int S, int KC, bool PULL>
__global__ void __launch_bounds__(256) k_pair_valu(PairArgs a, int64_t j_per_split,
                                                   double tau0, double tau1, double tau2, double tau3,
                                                   double tau4, double tau5, double kd0, double kd1,
                                                   double kd2, double kd3, double kd4, double kd5) {
  const double taud[6] = {tau0, tau1, tau2, tau3, tau4, tau5};
  const double kapd[6] = {kd0, kd1, kd2, kd3, kd4, kd5};
  pair_valu_body<S, KC, PULL>(a, j_per_split, taud, kapd, blockIdx.x, blockIdx.y);
}

// Many node sets (push form): block b takes work item items[b] = (set, block of 64 targets, source
// split), the same blocks as the single-run launch of that set.
template <int S, int KC>
__global__ void __launch_bounds__(256) k_pair_valu_batch(const ValuSet* __restrict__ sets,
                                                         const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const ValuSet& v = sets[it.x];
  pair_valu_body<S, KC, false>(v.a, v.per, v.taud, v.kapd, it.y, it.z);
}

int valu_kc(int32_t r) { return r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : 16; }

int64_t valu_per(const PairArgs& a) {
  const int64_t jtiles = (a.n + kVJ - 1) / kVJ;
  return ((jtiles + a.nsplit - 1) / a.nsplit) * kVJ;
}

template <int S>
static void launch_valu_batch_s(hipStream_t st, int kc, const ValuSet* sets, const int4* items, int nitems) {
  if (kc == 2) k_pair_valu_batch<S, 2><<<nitems, 256, 0, st>>>(sets, items);
  else if (kc == 4) k_pair_valu_batch<S, 4><<<nitems, 256, 0, st>>>(sets, items);
  else if (kc == 8) k_pair_valu_batch<S, 8><<<nitems, 256, 0, st>>>(sets, items);
  else k_pair_valu_batch<S, 16><<<nitems, 256, 0, st>>>(sets, items);
}

yy_status launch_pair_valu_batch(hipStream_t st, int32_t S, int kc, const ValuSet* sets, const int4* items,
                                 int nitems) {
  if (nitems <= 0) return YY_OK;
  switch (S) {
    case 1: launch_valu_batch_s<1>(st, kc, sets, items, nitems); break;
    case 2: launch_valu_batch_s<2>(st, kc, sets, items, nitems); break;
    case 3: launch_valu_batch_s<3>(st, kc, sets, items, nitems); break;
    case 4: launch_valu_batch_s<4>(st, kc, sets, items, nitems); break;
    case 5: launch_valu_batch_s<5>(st, kc, sets, items, nitems); break;
    case 6: launch_valu_batch_s<6>(st, kc, sets, items, nitems); break;
    default: return fail(YY_ERR_ARG, "bad scale count");
  }
  YY_LAUNCH_CHECK("k_pair_valu_batch");
  return YY_OK;
}

template <int S>
static yy_status launch_valu_s(hipStream_t st, const PairArgs& a, const double* taud,
                               const double* kapd) {
  const int64_t tiles = (a.n + kVI - 1) / kVI;
  const int64_t per = valu_per(a);
  dim3 grid((unsigned)tiles, (unsigned)a.nsplit);
#define YY_VALU_LAUNCH(KC)                                                                              \
  do {                                                                                                  \
    if (a.pull)                                                                                         \
      k_pair_valu<S, KC, true><<<grid, 256, 0, st>>>(a, per, taud[0], taud[1], taud[2], taud[3], taud[4], \
                                                     taud[5], kapd[0], kapd[1], kapd[2], kapd[3], kapd[4], \
                                                     kapd[5]);                                          \
    else                                                                                                \
      k_pair_valu<S, KC, false><<<grid, 256, 0, st>>>(a, per, taud[0], taud[1], taud[2], taud[3], taud[4], \
                                                      taud[5], kapd[0], kapd[1], kapd[2], kapd[3], kapd[4], \
                                                      kapd[5]);                                         \
  } while (0)
  const int kc = valu_kc(a.r);
  if (kc == 2) YY_VALU_LAUNCH(2);
  else if (kc == 4) YY_VALU_LAUNCH(4);
  else if (kc == 8) YY_VALU_LAUNCH(8);
  else YY_VALU_LAUNCH(16);
#undef YY_VALU_LAUNCH
  YY_LAUNCH_CHECK("k_pair_valu");
  return YY_OK;
}

static yy_status launch_pair_valu_d(hipStream_t st, const PairArgs& a, const double* taud,
                                    const double* kapd) {
  switch (a.S) {
    case 1: return launch_valu_s<1>(st, a, taud, kapd);
    case 2: return launch_valu_s<2>(st, a, taud, kapd);
    case 3: return launch_valu_s<3>(st, a, taud, kapd);
    case 4: return launch_valu_s<4>(st, a, taud, kapd);
    case 5: return launch_valu_s<5>(st, a, taud, kapd);
    case 6: return launch_valu_s<6>(st, a, taud, kapd);
  }
  return fail(YY_ERR_ARG, "bad scale count");
}

// ---------------------------------------------------------------------------
// Divergence of the drift at every node (the pull-form kernel's factor
// exp(-tau div f(x_i)), eq. kernel): closed form, or the complex-step sum of
// Sec. 8, sum_k Im f_k(x + i h e_k) / h, with complex arithmetic on (re, im)
// pairs: sin(a + i b) = sin a cosh b + i cos a sinh b, cos(a + i b) =
// cos a cosh b - i sin a sinh b.  One thread per node, FP64.
struct cplx {
  double re, im;
};
__device__ inline cplx c_mul(cplx u, cplx v) { return {u.re * v.re - u.im * v.im, u.re * v.im + u.im * v.re}; }
__device__ inline cplx c_sin(cplx z) { return {sin(z.re) * cosh(z.im), cos(z.re) * sinh(z.im)}; }
__device__ inline cplx c_cos(cplx z) { return {cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)}; }

__global__ void __launch_bounds__(kBlock) k_divergence(int64_t n, int32_t r, int32_t drift,
                                                       const double* __restrict__ A,
                                                       const double* __restrict__ x, int32_t mode, double h,
                                                       double* __restrict__ div) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double* xi = x + (size_t)i * r;
  double acc = 0.0;
  for (int32_t k = 0; k < r; ++k) {
    const double xk = xi[k], nxt = k + 1 < r ? xi[k + 1] : 0.0;
    if (drift == YY_F_ZERO) continue;
    if (mode == YY_DIV_COMPLEX_STEP) {
      const cplx z = {xk, h};
      cplx f;
      if (drift == YY_F_COS) {
        f = c_cos(z);
      } else if (drift == YY_F_PAPER_SINMIX) {
        const cplx z2 = {2.0 * xk, 2.0 * h};
        const cplx u = c_mul(c_sin(z), cplx{-0.5 * z.re + 0.1 * nxt, -0.5 * z.im});
        const cplx v = c_mul(c_sin(z2), cplx{-0.3 * z.re + 0.3 * nxt, -0.3 * z.im});
        f = {u.re + v.re, u.im + v.im};
      } else {   // linear: only the diagonal entry meets the imaginary step
        f = {0.0, A[(size_t)k * r + k] * h};
      }
      acc += f.im / h;
    } else if (drift == YY_F_COS) {
      acc += -sin(xk);
    } else if (drift == YY_F_PAPER_SINMIX) {
      acc += cos(xk) * (-0.5 * xk + 0.1 * nxt) - 0.5 * sin(xk) + 2.0 * cos(2.0 * xk) * (-0.3 * xk + 0.3 * nxt) -
             0.3 * sin(2.0 * xk);
    } else {
      acc += A[(size_t)k * r + k];
    }
  }
  div[i] = acc;
}

// ---------------------------------------------------------------------------
// (4) combination in FP64: merge the source splits, add the constants, signed
// log-sum-exp over the scales and the identity term.

// (the argument set by reference: in the batched kernel it lives in global memory, and a copy would be
// private memory on every lane)
__device__ __forceinline__ void k_combine_body(const CombineArgs& a, int bx_, int gx_) {
  const int64_t i = (int64_t)bx_ * kBlock + threadIdx.x;
  if (i >= a.n) return;
  // deferred planes: written in this call when the screen flagged a tile
  if (a.defer && i == 0 && a.defer[0]) a.defer[1] = 1;
  if (a.bnd[i]) {
    a.logw_out[i] = -INFINITY;
    return;
  }
  const double logvol = a.scal[0];
  const double lref = *a.lref;
  // no tile flagged in this call: every split keeps its starting state, (row floor, 0) except in
  // the split that holds the self pair, so that split's state alone gives the same (max, sum); it is
  // formed here (owner_start) and the split pass writes nothing
  const bool owner_only = a.defer && a.defer[0] == 0;
  const float li2 = owner_only ? a.lw2[i] : 0.f;
  const double fn = owner_only ? a.node[a.n + i] : 0.0;
  double T[YY_MAX_SCALES + 1], sg[YY_MAX_SCALES + 1];
  int nt = 0;
  for (int s = 0; s < a.S; ++s) {
    if (a.sign[s] == 0.0 || lref == -INFINITY) continue;
    float M = -INFINITY;
    double sum = 0.0;
    if (owner_only) {
      const float2 v = owner_start(li2, fn, a.kapd[s], a.taud[s], a.rref, a.rhv, a.n, i, s);
      M = v.x;
      if (M == -INFINITY) continue;
      sum = (double)v.y * exp2((double)v.x - (double)M);
    } else {
      for (int p = 0; p < a.nsplit; ++p) M = fmaxf(M, a.part[((size_t)p * a.S + s) * a.n + i].x);
      if (M == -INFINITY) continue;
      for (int p = 0; p < a.nsplit; ++p) {
        const float2 v = a.part[((size_t)p * a.S + s) * a.n + i];
        if (v.x != -INFINITY) sum += (double)v.y * exp2((double)v.x - (double)M);
      }
    }
    const double L = ((double)M + log2(sum)) * kLn2 + lref;
    T[nt] = a.kap[s] + logvol + L;
    if (a.div) T[nt] -= a.taud[s] * a.div[i];   // pull form: exp(-tau_s div f(x_i))
    sg[nt] = a.sign[s];
    ++nt;
  }
  const double li = a.logw_in[i];
  if (a.sign[a.S] != 0.0 && li != -INFINITY) {
    T[nt] = a.logc_id + li;
    sg[nt] = a.sign[a.S];
    ++nt;
  }
  if (nt == 0) {
    a.logw_out[i] = -INFINITY;
    return;
  }
  double Mx = T[0];
  for (int t = 1; t < nt; ++t) Mx = fmax(Mx, T[t]);
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) acc += sg[t] * exp(T[t] - Mx);
  if (!(acc > 0.0)) {
    a.logw_out[i] = -INFINITY;
    atomicOr(a.flags, YY_FLAG_CLAMPED);
    atomicAdd(a.nclamped, 1ULL);
    return;
  }
  a.logw_out[i] = Mx + log(acc);
}

__global__ void __launch_bounds__(kBlock) k_combine(CombineArgs a) {
  k_combine_body(a, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_combine_batch(const combine_args* __restrict__ A,
                                                          const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const combine_args& a = A[q];
  if (a.pred && *a.pred == 0) return;
  k_combine_body(a.a, blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


// ---------------------------------------------------------------------------
// K of the prepared node set: r zero-padded to whole groups of 16-wide K
// stages of the pairwise kernel (2 stages per barrier; 4 for BF16X1, the
// vector-ALU form and the screens of BF16X3S and BF16X3P at r > 256, where the
// padding to 64 costs at most a few percent).
int pair_mfma_rp(int32_t r, int32_t prec) {
  const bool screened = prec == YY_PREC_BF16X3S || prec == YY_PREC_BF16X3P;
  const int q = (prec == YY_PREC_BF16X1 || prec == YY_PREC_FP32 || (screened && r > 256)) ? 64 : 32;
  return ((r + q - 1) / q) * q;
}

yy_status prepare_nodes(yy_ctx ctx, const yy_model* m, int64_t n, const double* x,
                        uint64_t version, const double* lo, const double* hi, bool want_bf16,
                        bool want_f32t, int32_t prec, bool defer_planes) {
  Prepared& P = ctx->prep;
  // general process noise: the kernels run on the whitened coordinates W (x - c), W f(x) (k of them)
  const bool white = noise_a(m);
  const int32_t rk = white ? m->noise->rank_a : m->r;
  const int32_t rp = pair_mfma_rp(rk, prec);
  const bool defer = defer_planes && prec == YY_PREC_BF16X3P && want_bf16 && !want_f32t && !white;
  const bool same = P.valid && P.x == x && P.n == n && P.r == m->r && P.rp == rp && P.drift == m->drift &&
                    P.A == m->A && P.version == version && P.lo == lo && P.hi == hi &&
                    (P.have_bf16 || !want_bf16) && (P.have_f32t || !want_f32t) && (!P.deferred || defer) &&
                    P.noise == (const void*)(white ? m->noise : nullptr);
  if (same) return YY_OK;
  P.div_mode = -1;
  const int64_t n_pad = pair_mfma_npad(n);
  yy_status st;
  if ((st = P.xc32.ensure((size_t)n * rp * sizeof(float))) != YY_OK) return st;
  if ((st = P.f32.ensure((size_t)n * rp * sizeof(float))) != YY_OK) return st;
  if (want_bf16 && (st = P.bf.ensure((size_t)4 * n_pad * rp * sizeof(uint16_t))) != YY_OK) return st;
  if (want_f32t && (st = P.f32t.ensure((size_t)2 * n_pad * rp * sizeof(float))) != YY_OK) return st;
  const int nparts = prepare_blocks(n_pad);
  if ((st = P.node.ensure(((size_t)6 * n + 4 * (size_t)nparts) * sizeof(double))) != YY_OK) return st;
  if ((st = P.bnd.ensure((size_t)n * sizeof(int))) != YY_OK) return st;
  if ((st = P.scal.ensure(8 * sizeof(double))) != YY_OK) return st;
  WhiteNodes wn{};
  if (white && (st = noise_whiten_nodes(ctx, m, n, x, lo, hi, wn)) != YY_OK) return st;
  // the whitened coordinates are centred already: a zero box centre, the boundary flags given
  const double* px = white ? wn.x : x;
  const double* plo = white ? wn.zeros : lo;
  const double* phi = white ? wn.zeros : hi;
  const int32_t pdrift = white ? kDriftGiven : m->drift;
  if (defer) {
    k_prepare<1><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
        n, n_pad, m->r, rp, m->drift, m->A, x, lo, hi, nullptr, nullptr, P.bf.as<uint16_t>(), nullptr,
        P.node.as<double>(), P.bnd.as<int>(), ctx->d_defer, nullptr, nullptr);
  } else {
    k_prepare<0><<<(unsigned)nparts, kBlock, 0, ctx->stream>>>(
        n, n_pad, rk, rp, pdrift, m->A, px, plo, phi, P.xc32.as<float>(), P.f32.as<float>(),
        want_bf16 ? P.bf.as<uint16_t>() : nullptr, want_f32t ? P.f32t.as<float>() : nullptr,
        P.node.as<double>(), P.bnd.as<int>(), nullptr, white ? wn.f : nullptr, white ? wn.bnd : nullptr);
  }
  YY_LAUNCH_CHECK("k_prepare");
  // (the box volume from the original box)
  k_prepare_scalars<<<1, kBlock, 0, ctx->stream>>>(n, m->r, nparts, lo, hi, P.node.as<double>(),
                                                   P.scal.as<double>());
  YY_LAUNCH_CHECK("k_prepare_scalars");
  P.valid = true;
  P.x = x;
  P.n = n;
  P.n_pad = n_pad;
  P.r = m->r;
  P.rp = rp;
  P.drift = m->drift;
  P.A = m->A;
  P.version = version;
  P.lo = lo;
  P.hi = hi;
  P.have_bf16 = want_bf16;
  P.have_f32t = want_f32t;
  P.deferred = defer;
  P.noise = white ? m->noise : nullptr;
  P.dp = DeferredPrep{n, n_pad, m->r, rp, m->drift, m->A, x, lo, hi, P.xc32.as<float>(), P.f32.as<float>(),
                      P.bf.as<uint16_t>(), ctx->d_defer};
  return YY_OK;
}

static yy_status check_model(const yy_model* m) {
  if (!m) return fail(YY_ERR_ARG, "model is NULL");
  if (m->r < 1 || m->r > YY_MAX_R) return fail(YY_ERR_ARG, "model r out of range");
  if (m->drift < YY_F_ZERO || m->drift > YY_F_PAPER_SINMIX) return fail(YY_ERR_ARG, "unknown drift");
  if (m->drift == YY_F_LINEAR && !m->A) return fail(YY_ERR_ARG, "linear drift needs A");
  if (m->obs < YY_H_IDENTITY || m->obs > YY_H_LINEAR) return fail(YY_ERR_ARG, "unknown observation");
  if (m->obs == YY_H_LINEAR && !m->H) return fail(YY_ERR_ARG, "linear observation needs H");
  if (m->obs != YY_H_LINEAR && m->m != m->r) return fail(YY_ERR_ARG, "m must equal r for this h");
  if (m->m < 1) return fail(YY_ERR_ARG, "m must be positive");
  if (!(m->q > 0.0) || !(m->rho2 > 0.0)) return fail(YY_ERR_ARG, "noise variances must be positive");
  if (m->noise) {
    if (m->noise->rank_a > 0 && m->noise->r != m->r) return fail(YY_ERR_ARG, "noise: U is not r x r");
    if (m->noise->rank_b > 0 && m->noise->m != m->m) return fail(YY_ERR_ARG, "noise: V is not m x m");
  }
  return YY_OK;
}

yy_status validate_model(const yy_model* m) { return check_model(m); }


// Host launchers of the batched kernels (one block range per argument set).
yy_status launch_batched(hipStream_t st, const prepare_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_prepare_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_prepare_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const prepare_scalars_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_prepare_scalars_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_prepare_scalars_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const lw_max_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_lw_max_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_lw_max_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const lw_convert_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_lw_convert_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_lw_convert_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const RowRefArgs* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_heavy_batch<<<nr, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_heavy_batch");
  k_row_ref_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_row_ref_batch");
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const combine_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_combine_batch<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_combine_batch");
  return YY_OK;
}

}  // namespace yy

using namespace yy;

namespace yy {

// Source weights relative to their maximum (step 2): lw2 [n] and the device
// address of the maximum (in ctx->red).
yy_status source_weights(yy_ctx ctx, int64_t n, const double* logw_in, const int* bnd, float* lw2,
                         double** lref_out, long long** heavy_out) {
  const int nparts = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  yy_status st;
  if ((st = ctx->red.ensure((size_t)(2 * nparts + 8) * sizeof(double))) != YY_OK) return st;
  double* d_part = ctx->red.as<double>();
  double* d_lref = d_part + nparts;
  // [nparts + 1]: j* (k_heavy); [nparts + 8 ..]: the conversion blocks' candidates
  long long* d_heavy = reinterpret_cast<long long*>(d_part + nparts + 8);
  if (heavy_out) *heavy_out = d_heavy;
  k_lw_max<<<nparts, kBlock, 0, ctx->stream>>>(n, logw_in, bnd, d_part);
  YY_LAUNCH_CHECK("k_lw_max");
  k_lw_convert<<<nparts, kBlock, 0, ctx->stream>>>(n, nparts, d_part, logw_in, bnd, lw2, d_lref,
                                                   heavy_out ? d_heavy : nullptr);
  YY_LAUNCH_CHECK("k_lw_convert");
  *lref_out = d_lref;
  return YY_OK;
}

yy_status launch_combine(hipStream_t st, const CombineArgs& cb) {
  if (cb.n == 0) return YY_OK;
  k_combine<<<(unsigned)((cb.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(cb);
  YY_LAUNCH_CHECK("k_combine");
  return YY_OK;
}

// Steps (1), (2) and the launch parameters of (3) and (4) for one call; the
// batched step (yy_batch.hip) runs (3) for many plans in one launch.
std::vector<int4> sym_work_items(int64_t tbs) {
  std::vector<int4> items;
  for (int64_t A = 0; A < tbs; ++A)
    for (int64_t B0 = A; B0 < tbs; B0 += kSymChunk)
      items.push_back(make_int4((int)A, (int)B0, (int)std::min<int64_t>(B0 + kSymChunk, tbs), 0));
  std::stable_sort(items.begin(), items.end(), [](const int4& u, const int4& v) {
    const int lu = u.z - u.y, lv = v.z - v.y;
    return lu != lv ? lu > lv : u.y < v.y;
  });
  return items;
}

yy_status propagate_begin(yy_ctx ctx, const yy_model* model, const yy_scales* scales, int32_t prec, int64_t n,
                          const double* x, uint64_t node_version, const double* box_lo, const double* box_hi,
                          double dt, const double* logw_in, double* logw_out, int nsplit_override,
                          PropPlan& plan, bool defer_planes) {
  yy_status st = check_model(model);
  if (st != YY_OK) return st;
  if (!scales || scales->S < 1 || scales->S > YY_MAX_SCALES || !scales->s)
    return fail(YY_ERR_ARG, "yy_propagate: bad scales");
  if (n < 0) return fail(YY_ERR_ARG, "yy_propagate: n < 0");
  if (n > ((int64_t)1 << 31)) return fail(YY_ERR_UNSUPPORTED, "yy_propagate: n above 2^31");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(YY_ERR_ARG, "yy_propagate: dt must be positive");
  plan.n = n;
  if (n == 0) return YY_OK;
  if (!x || !box_lo || !box_hi || !logw_in || !logw_out)
    return fail(YY_ERR_ARG, "yy_propagate: NULL array");
  if (logw_in == logw_out) return fail(YY_ERR_ARG, "yy_propagate: logw_in and logw_out alias");
  if (prec < YY_PREC_AUTO || prec > YY_PREC_BF16X3P) return fail(YY_ERR_ARG, "yy_propagate: bad prec");
  const int32_t S = scales->S;
  double c[YY_MAX_SCALES + 1];
  for (int s = 0; s < S; ++s)
    if (!(scales->s[s] > 0.0)) return fail(YY_ERR_ARG, "yy_propagate: scale divisors must be > 0");
  if (scales->c) {
    for (int s = 0; s <= S; ++s) c[s] = scales->c[s];
  } else if ((st = coefficients_cramer(S, scales->s, c)) != YY_OK) {
    return st;
  }
  const int32_t r = model->r;
  if (prec == YY_PREC_AUTO) prec = r < 32 ? YY_PREC_FP32 : YY_PREC_BF16X3;
  const bool mfma = prec != YY_PREC_FP32;
  if (scales->form != YY_FORM_PUSH && scales->form != YY_FORM_PULL)
    return fail(YY_ERR_ARG, "yy_propagate: unknown kernel form");
  const bool pull = scales->form == YY_FORM_PULL;
  if (pull && scales->div != YY_DIV_CLOSED && scales->div != YY_DIV_COMPLEX_STEP)
    return fail(YY_ERR_ARG, "yy_propagate: unknown divergence mode");
  if (pull && (prec == YY_PREC_BF16X3S || prec == YY_PREC_BF16X3P))
    return fail(YY_ERR_UNSUPPORTED, "yy_propagate: the screened forms are push-form only");
  if (mfma && S > 4) return fail(YY_ERR_UNSUPPORTED, "the matrix-core path supports up to 4 scales");
  plan.prec = prec;
  plan.mfma = mfma;
  YY_HIP(hipSetDevice(ctx->device));
  st = prepare_nodes(ctx, model, n, x, node_version, box_lo, box_hi,
                     prec == YY_PREC_BF16X3 || prec == YY_PREC_BF16X3G || prec == YY_PREC_BF16X1 ||
                         prec == YY_PREC_BF16X3S || prec == YY_PREC_BF16X3P,
                     prec == YY_PREC_FP32_MFMA, prec, defer_planes);
  if (st != YY_OK) return st;
  Prepared& P = ctx->prep;
  if (pull && P.div_mode != scales->div) {
    // the divergence of f at every node, once per node set and mode
    if ((st = P.div.ensure((size_t)n * sizeof(double))) != YY_OK) return st;
    k_divergence<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        n, r, model->drift, model->A, x, scales->div, 1e-20, P.div.as<double>());
    YY_LAUNCH_CHECK("k_divergence");
    P.div_mode = scales->div;
  }

  // (2) source weights relative to their maximum
  if ((st = ctx->lw2.ensure((size_t)n * sizeof(float))) != YY_OK) return st;
  double* d_lref = nullptr;
  long long* d_heavy = nullptr;
  if ((st = source_weights(ctx, n, logw_in, P.bnd.as<int>(), ctx->lw2.as<float>(), &d_lref, &d_heavy)) != YY_OK)
    return st;

  // (3) pairwise partials
  PairArgs& a = plan.a;
  a = PairArgs{};
  const bool white = noise_a(model);
  const double qk = white ? 1.0 : model->q;   // the whitened coordinates have unit variance per unit time
  a.n = n;
  a.r = white ? model->noise->rank_a : r;
  a.rp = P.rp;
  a.S = S;
  a.pull = pull ? 1 : 0;
  double taud[6] = {0, 0, 0, 0, 0, 0}, kapd[6] = {0, 0, 0, 0, 0, 0};
  for (int s = 0; s < S; ++s) {
    taud[s] = dt / scales->s[s];
    kapd[s] = kLog2e / (2.0 * qk * taud[s]);
    a.tau[s] = (float)taud[s];
    a.kap2[s] = (float)kapd[s];
    plan.taud[s] = taud[s];
    plan.kapd[s] = kapd[s];
  }
  a.xc = P.xc32.as<float>();
  a.f = P.f32.as<float>();
  a.lw2 = ctx->lw2.as<float>();
  a.node = P.node.as<double>();
  a.bnd = P.bnd.as<int>();
  a.bf = P.have_bf16 ? P.bf.as<uint16_t>() : nullptr;
  a.scal = P.scal.as<double>();
  // enough blocks to cover the chip: split the source range when targets are few
  const int64_t ttiles = (n + kVI - 1) / kVI;
  int nsplit = 1;
  MfmaExtra& ex = plan.ex;
  ex = MfmaExtra{};
  if (mfma) {
    // the matrix-core kernel: 256-target blocks, 128-source tiles.  16 source
    // splits let one XCD (32 CUs, one block each) work on 2 target blocks at a
    // time; small problems split further until 256 blocks cover the chip.  A
    // tuned split count (yy_tune) or the caller's override replaces the rule.
    const int64_t n_pad = P.n_pad, tbs = n_pad / 256, jtl = (n + 127) / 128;
    const int tuned = tune_lookup(ctx, P.rp, n_pad, S, prec);
    if (nsplit_override > 0) {
      nsplit = nsplit_override;
    } else if (tuned > 0) {
      nsplit = tuned;
    } else {
      nsplit = 16;
      while (tbs * nsplit < 256 && nsplit < 256) nsplit *= 2;
    }
    if (nsplit > jtl) nsplit = (int)jtl;
    ex.n_pad = n_pad;
    ex.f32t = P.have_f32t ? P.f32t.as<float>() : nullptr;
    ex.j_per_split = ((jtl + nsplit - 1) / nsplit) * 128;
    nsplit = (int)((jtl * 128 + ex.j_per_split - 1) / ex.j_per_split);
    for (int s = 0; s < S; ++s) {
      ex.kapd[s] = kapd[s];
      ex.taud[s] = taud[s];
    }
    // (BF16X3P: the biases over the first kPreK coordinates follow in the same layout)
    const size_t bsz = (size_t)S * (n_pad + n_pad / 128);
    if ((st = ctx->bsrc.ensure((prec == YY_PREC_BF16X3P ? 2 : 1) * bsz * sizeof(float))) != YY_OK) return st;
    ex.bsrc = ctx->bsrc.as<float>();
    ex.bpre = prec == YY_PREC_BF16X3P ? ex.bsrc + bsz : nullptr;
    ex.deferred = P.deferred ? &P.dp : nullptr;
    if (prec == YY_PREC_BF16X3S || prec == YY_PREC_BF16X3P) {
      if ((st = ctx->sflags.ensure((size_t)tbs * jtl * 8)) != YY_OK) return st;
      ex.flags = ctx->sflags.as<uint8_t>();
      ctx->sflags_tbs = tbs;
      ctx->sflags_jtl = jtl;
    }
  } else {
    while (ttiles * nsplit < 512 && nsplit < 64 && (int64_t)nsplit * kVJ * 2 <= n) nsplit *= 2;
  }
  a.nsplit = nsplit;
  if ((st = ctx->part.ensure((size_t)nsplit * S * n * sizeof(float2))) != YY_OK) return st;
  a.part = ctx->part.as<float2>();
  if (mfma && pull && (st = launch_src_bias(ctx->stream, a, ex)) != YY_OK) return st;
  if (mfma && !pull) {
    // a lower bound of every row maximum: the self pair, or the pair with the heaviest source
    if ((st = ctx->rref.ensure(2 * (size_t)S * n * sizeof(float))) != YY_OK) return st;
    RowRefArgs ra{};
    ra.n = n;
    ra.r = a.r;
    ra.S = S;
    ra.drift = model->drift;
    ra.A = model->A;
    ra.x = white ? static_cast<const double*>(P.wnodes.ptr) : x;
    ra.fw = white ? static_cast<const double*>(P.wnodes.ptr) + (size_t)n * a.r : nullptr;
    ra.lw2 = a.lw2;
    ra.node = a.node;
    ra.bnd = a.bnd;
    ra.heavy = d_heavy;
    ra.nheavy = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    ra.jstar = reinterpret_cast<long long*>(d_lref + 1);
    if ((st = ctx->fstar.ensure((size_t)a.r * sizeof(double))) != YY_OK) return st;
    ra.fstar = ctx->fstar.as<double>();
    for (int s = 0; s < S; ++s) {
      ra.kapd[s] = kapd[s];
      ra.taud[s] = taud[s];
    }
    ra.rref = ctx->rref.as<float>();
    ra.rhv = ra.rref + (size_t)S * n;
    // the source biases and j* (with f(x_j*)) in one launch: both read only the converted weights
    if ((st = launch_src_bias_heavy(ctx->stream, a, ex, ra)) != YY_OK) return st;
    k_row_ref<<<(unsigned)((n + row_ref_targets(a.r, n) - 1) / row_ref_targets(a.r, n)), kBlock, 0, ctx->stream>>>(ra);
    YY_LAUNCH_CHECK("k_row_ref");
    ex.rref = ra.rref;
    ex.rhv = ra.rhv;
    ex.jstar = ra.jstar;
    const int64_t tbs = ex.n_pad / 256;
    // (only where the screen spans 64 coordinates: over 32 the transposed coarse bound leaves most groups
    // in doubt, and their rechecks cost more than the halved products save)
    if (prec == YY_PREC_BF16X3P && tbs > kSymMinBlocks && a.rp > 32) {
      // the symmetric screen's work items: target block A against the target blocks [B0, B1) >= A as
      // sources, kSymChunk at a time, the longest first (then by source range, so that items started
      // together share sources); built once per block count
      if (ctx->sym_tbs != tbs) {
        const std::vector<int4> items = sym_work_items(tbs);
        if ((st = ctx->sym_items.ensure(items.size() * sizeof(int4))) != YY_OK) return st;
        YY_HIP(hipMemcpyAsync(ctx->sym_items.ptr, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice,
                              ctx->stream));
        YY_HIP(hipStreamSynchronize(ctx->stream));   // `items` is a host temporary
        int64_t tiles = 0;
        for (const int4& u : items) tiles += 2 * (int64_t)(u.z - u.y);
        ctx->sym_tbs = tbs;
        ctx->sym_nitems = (int)items.size();
        ctx->sym_cap = (int)std::min<int64_t>(8 * tiles, kSymListMax);
      }
      if ((st = ctx->tT.ensure(2 * (size_t)S * (ex.n_pad / 64) * sizeof(float))) != YY_OK) return st;
      if ((st = ctx->sym_list.ensure(16 + (size_t)ctx->sym_cap * sizeof(int4))) != YY_OK) return st;
      ex.sym_items = ctx->sym_items.as<int4>();
      ex.tT = ctx->tT.as<float>();
      ex.sym_nitems = ctx->sym_nitems;
      ex.sym_n = ctx->sym_list.as<int>();
      ex.sym_list = reinterpret_cast<int4*>(ctx->sym_list.as<unsigned char>() + 16);
      ex.sym_cap = ctx->sym_cap;
    }
  }

  // (4) combination parameters
  CombineArgs& cb = plan.cb;
  cb = CombineArgs{};
  cb.n = n;
  cb.S = S;
  cb.nsplit = a.nsplit;
  for (int s = 0; s < S; ++s) {
    // Gaussian constant: (2 pi q tau)^{-r/2}, or (2 pi tau)^{-r/2} det_+(a)^{-1/2} for general noise
    cb.kap[s] = (c[s] != 0.0 ? std::log(std::fabs(c[s])) : 0.0) - std::log((double)n) -
                (white ? 0.5 * r * std::log(2.0 * M_PI * taud[s]) + 0.5 * model->noise->logdet_a
                       : 0.5 * r * std::log(2.0 * M_PI * model->q * taud[s]));
    cb.sign[s] = c[s] > 0 ? 1.0 : (c[s] < 0 ? -1.0 : 0.0);
  }
  cb.sign[S] = c[S] > 0 ? 1.0 : (c[S] < 0 ? -1.0 : 0.0);
  cb.logc_id = c[S] != 0.0 ? std::log(std::fabs(c[S])) : 0.0;
  cb.part = a.part;
  cb.scal = P.scal.as<double>();
  cb.lref = d_lref;
  cb.logw_in = logw_in;
  cb.bnd = P.bnd.as<int>();
  cb.logw_out = logw_out;
  cb.flags = ctx->d_flags;
  cb.nclamped = ctx->d_nclamped;
  cb.defer = P.deferred && mfma ? ctx->d_defer : nullptr;
  cb.j_per_split = ex.j_per_split;
  cb.div = pull ? P.div.as<double>() : nullptr;
  for (int s = 0; s < S; ++s) {
    cb.taud[s] = taud[s];
    cb.kapd[s] = kapd[s];
  }
  cb.lw2 = a.lw2;
  cb.node = a.node;
  cb.rref = mfma && !pull ? ex.rref : nullptr;
  cb.rhv = mfma && !pull ? ex.rhv : nullptr;
  return YY_OK;
}

yy_status propagate_pair(yy_ctx ctx, const PropPlan& plan) {
  if (plan.n == 0) return YY_OK;
  yy_status st;
  if ((st = timing_begin(ctx)) != YY_OK) return st;
  if (plan.mfma) {
    st = launch_pair_mfma(ctx->stream, plan.a, plan.prec, plan.ex);
  } else {
    st = launch_pair_valu_d(ctx->stream, plan.a, plan.taud, plan.kapd);
  }
  if (st != YY_OK) return st;
  return timing_end(ctx);
}

yy_status propagate_end(yy_ctx ctx, const PropPlan& plan) {
  if (plan.n == 0) return YY_OK;
  return launch_combine(ctx->stream, plan.cb);
}

}  // namespace yy

extern "C" yy_status yy_propagate(yy_ctx ctx, const yy_model* model, const yy_scales* scales,
                                  int32_t prec, int64_t n, const double* x, uint64_t node_version,
                                  const double* box_lo, const double* box_hi, double dt,
                                  const double* logw_in, double* logw_out) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_propagate: ctx is NULL");
  PropPlan plan;
  yy_status st = propagate_begin(ctx, model, scales, prec, n, x, node_version, box_lo, box_hi, dt, logw_in,
                                 logw_out, 0, plan, true);
  if (st != YY_OK) return st;
  if ((st = propagate_pair(ctx, plan)) != YY_OK) return st;
  return propagate_end(ctx, plan);
}

extern "C" yy_status yy_screen_count(yy_ctx ctx, int64_t* flagged, int64_t* tiles) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_screen_count: ctx is NULL");
  if (!flagged || !tiles) return fail(YY_ERR_ARG, "yy_screen_count: NULL output");
  if (ctx->sflags_tbs <= 0) return fail(YY_ERR_ARG, "yy_screen_count: no screened propagation on this context");
  YY_HIP(hipSetDevice(ctx->device));
  YY_HIP(hipStreamSynchronize(ctx->stream));
  const int64_t t = ctx->sflags_tbs * ctx->sflags_jtl;
  std::vector<uint64_t> h((size_t)t);
  YY_HIP(hipMemcpy(h.data(), ctx->sflags.ptr, (size_t)t * 8, hipMemcpyDeviceToHost));
  int64_t c = 0;
  for (uint64_t v : h) c += v != 0;
  *flagged = c;
  *tiles = t;
  return YY_OK;
}
