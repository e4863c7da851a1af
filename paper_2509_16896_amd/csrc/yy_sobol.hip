// yy_sobol.hip -- Sobol node generation (Appendix A, Sobol sequence) and the
// code -> box map shared by initial sampling and the Sec. 6 restart.
#include "yy_internal.h"

namespace yy {

// One thread per (point, dimension), dimension fastest so stores are coalesced.
// code = shift ^ xor_{k : bit k of gray(i)} v'_k, with v' the scrambled table.
__global__ void __launch_bounds__(kBlock) k_sobol(int32_t r, int64_t n, uint64_t first,
                                                  const uint32_t* __restrict__ table,
                                                  const double* __restrict__ lo,
                                                  const double* __restrict__ hi,
                                                  uint32_t* __restrict__ codes,
                                                  double* __restrict__ x) {
#pragma clang fp contract(off)
  const int64_t total = n * (int64_t)r;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / r;
    const int32_t d = (int32_t)(t - i * r);
    const uint64_t idx = first + (uint64_t)i;
    uint32_t g = (uint32_t)(idx ^ (idx >> 1));
    const uint32_t* v = table + (size_t)d * 33;
    uint32_t code = v[32];
    while (g) {
      const int k = __builtin_ctz(g);
      code ^= v[k];
      g &= g - 1u;
    }
    if (codes) codes[t] = code;
    if (x) {
      const double c = __dmul_rn(0.5, __dadd_rn(lo[d], hi[d]));
      const double hw = __dmul_rn(0.5, __dsub_rn(hi[d], lo[d]));
      const double u = __dsub_rn((double)code * 0x1p-31, 1.0);
      x[t] = __dadd_rn(c, __dmul_rn(hw, u));
    }
  }
}

static int grid_for(int64_t total) {
  int64_t g = (total + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_nodes_sobol(yy_ctx ctx, int32_t r, int64_t n, int64_t first_index,
                                    int32_t scramble, uint64_t seed, const double* box_lo,
                                    const double* box_hi, uint32_t* codes, double* x) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_nodes_sobol: ctx is NULL");
  if (r < 1 || r > YY_MAX_R) return fail(YY_ERR_ARG, "yy_nodes_sobol: r out of range");
  if (n < 0 || first_index < 0 || (uint64_t)first_index + (uint64_t)n > (1ULL << 32))
    return fail(YY_ERR_ARG, "yy_nodes_sobol: point indices must lie in [0, 2^32)");
  if (x && (!box_lo || !box_hi)) return fail(YY_ERR_ARG, "yy_nodes_sobol: x needs box_lo/box_hi");
  if (n == 0 || (!codes && !x)) return YY_OK;
  YY_HIP(hipSetDevice(ctx->device));
  yy_status st = sobol_prepare_dirs(ctx, r, scramble ? 1 : 0, seed);
  if (st != YY_OK) return st;
  k_sobol<<<grid_for(n * (int64_t)r), kBlock, 0, ctx->stream>>>(
      r, n, (uint64_t)first_index, ctx->d_dirs.as<uint32_t>(), box_lo, box_hi, codes, x);
  YY_LAUNCH_CHECK("k_sobol");
  return YY_OK;
}
