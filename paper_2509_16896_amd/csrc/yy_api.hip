// yy_api.hip -- context management, argument checks and host-side set-up of libyy.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "yy_internal.h"

namespace yy {

static thread_local std::string g_last_error;

yy_status fail(yy_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

yy_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return YY_ERR_HIP;
}

yy_status DevBuf::ensure(size_t want) {
  if (want <= bytes && ptr) return YY_OK;
  if (ptr) {
    hipError_t e = hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  size_t alloc = want < 256 ? 256 : want;
  hipError_t e = hipMalloc(&ptr, alloc);
  if (e != hipSuccess) {
    ptr = nullptr;
    return fail(YY_ERR_ALLOC, "hipMalloc of " + std::to_string(alloc) + " bytes failed");
  }
  bytes = alloc;
  return YY_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// ---------------------------------------------------------------------------
// Sobol direction numbers (Appendix A).  Primitive polynomials of degree s are
// found by running the linear feedback shift register x -> x*t mod P from 1
// and checking that it first returns to 1 after exactly 2^s - 1 steps.

static const uint64_t kDirSeed = 0x59A0D1CE5EED0001ULL;  // key of the initial direction numbers
static const uint64_t kDomainScramble = 1ULL;

static uint64_t sm64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static bool lfsr_full_period(uint32_t poly, int deg) {
  const uint32_t period = (1u << deg) - 1u;
  uint32_t state = 1u;
  for (uint32_t step = 1; step <= period; ++step) {
    state <<= 1;
    if (state & (1u << deg)) state ^= poly;
    if (state == 1u) return step == period;
  }
  return false;
}

static void extend_dirs(yy_ctx ctx, int32_t r) {
  if (r <= ctx->dir_r) return;
  std::vector<uint32_t> polys;
  std::vector<int> degs;
  polys.reserve(r);
  for (int deg = 1; (int)polys.size() < r - 1; ++deg)
    for (uint32_t mid = 0; mid < (1u << (deg - 1)) && (int)polys.size() < r - 1; ++mid) {
      uint32_t p = (1u << deg) | (mid << 1) | 1u;
      if (lfsr_full_period(p, deg)) {
        polys.push_back(p);
        degs.push_back(deg);
      }
    }
  ctx->dirs.assign((size_t)r * 32, 0u);
  for (int32_t d = 0; d < r; ++d) {
    uint64_t m[33];
    if (d == 0) {
      for (int k = 1; k <= 32; ++k) m[k] = 1;
    } else {
      const uint32_t p = polys[d - 1];
      const int s = degs[d - 1];
      const uint64_t key = sm64(kDirSeed, (uint64_t)d);
      for (int k = 1; k <= s; ++k) m[k] = (sm64(key, (uint64_t)(k - 1)) >> (64 - k)) | 1ULL;
      for (int k = s + 1; k <= 32; ++k) {
        // Bratley-Fox recurrence: the polynomial's coefficient of t^{s-l} multiplies m_{k-l} 2^l.
        uint64_t v = m[k - s] ^ (m[k - s] << s);
        for (int l = 1; l < s; ++l)
          if ((p >> (s - l)) & 1u) v ^= m[k - l] << l;
        m[k] = v;
      }
    }
    for (int k = 1; k <= 32; ++k) ctx->dirs[(size_t)d * 32 + (k - 1)] = (uint32_t)(m[k] << (32 - k));
  }
  ctx->dir_r = r;
}

// The random linear scramble is applied to the direction numbers: scrambling
// is linear over GF(2), so L (xor_k v_k) = xor_k (L v_k), and the digital shift
// is xored once per point.  Table layout per dimension: 32 words + the shift.
yy_status sobol_prepare_dirs(yy_ctx ctx, int32_t r, int32_t scramble, uint64_t seed) {
  if (ctx->d_dirs_r >= r && ctx->d_dirs_scramble == scramble && (!scramble || ctx->d_dirs_seed == seed))
    return YY_OK;
  extend_dirs(ctx, r);
  std::vector<uint32_t> table((size_t)r * 33, 0u);
  for (int32_t d = 0; d < r; ++d) {
    const uint32_t* v = &ctx->dirs[(size_t)d * 32];
    uint32_t* out = &table[(size_t)d * 33];
    if (!scramble) {
      for (int k = 0; k < 32; ++k) out[k] = v[k];
      out[32] = 0;
      continue;
    }
    const uint64_t key = sm64(sm64(seed, kDomainScramble), (uint64_t)d);
    uint32_t rows[32];
    for (int p = 31; p >= 0; --p) {
      uint64_t rnd = sm64(key, (uint64_t)(31 - p)) >> 32;
      rows[p] = (uint32_t)(((rnd >> p) << p) | (1ULL << p));
    }
    for (int k = 0; k < 32; ++k) {
      uint32_t w = 0;
      for (int p = 0; p < 32; ++p) w |= (uint32_t)(__builtin_popcount(rows[p] & v[k]) & 1) << p;
      out[k] = w;
    }
    out[32] = (uint32_t)(sm64(key, 32) >> 32);
  }
  yy_status st = ctx->d_dirs.ensure(table.size() * sizeof(uint32_t));
  if (st != YY_OK) return st;
  YY_HIP(hipMemcpyAsync(ctx->d_dirs.ptr, table.data(), table.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice, ctx->stream));
  YY_HIP(hipStreamSynchronize(ctx->stream));  // `table` is a host temporary
  ctx->d_dirs_r = r;
  ctx->d_dirs_scramble = scramble;
  ctx->d_dirs_seed = seed;
  return YY_OK;
}

// ---------------------------------------------------------------------------
// Cramer's rule for V c = d (Sec. 4.3.3): c_j = det V_j / det V, determinants
// by the Leibniz permutation expansion (S + 1 <= 7 columns).
static double det_leibniz(const double* M, int N) {
  int perm[8];
  for (int i = 0; i < N; ++i) perm[i] = i;
  double total = 0.0;
  // Heap's algorithm over all permutations, tracking the sign.
  int c[8] = {0};
  int sign = 1;
  auto term = [&]() {
    double p = 1.0;
    for (int i = 0; i < N; ++i) p *= M[i * N + perm[i]];
    return sign * p;
  };
  total += term();
  int i = 0;
  while (i < N) {
    if (c[i] < i) {
      int a = (i % 2 == 0) ? 0 : c[i];
      int t = perm[a];
      perm[a] = perm[i];
      perm[i] = t;
      sign = -sign;
      total += term();
      ++c[i];
      i = 0;
    } else {
      c[i] = 0;
      ++i;
    }
  }
  return total;
}

yy_status coefficients_cramer(int32_t S, const double* s, double* c) {
  const int N = S + 1;
  double V[49], d[7];
  for (int col = 0; col < N; ++col) V[0 * N + col] = 1.0;
  d[0] = 1.0;
  for (int col = 0; col < N; ++col) V[1 * N + col] = col < S ? 1.0 / s[col] : 0.0;
  d[1] = 1.0;
  for (int k = 1; k <= S - 1; ++k) {
    const double mu = 0.5 * (k + 2);  // the paper's example exponents 3/2, 2, ...
    for (int col = 0; col < N; ++col) V[(1 + k) * N + col] = col < S ? std::pow(s[col], -mu) : 0.0;
    d[1 + k] = 0.0;
  }
  const double detV = det_leibniz(V, N);
  if (!(std::fabs(detV) > 0.0)) return fail(YY_ERR_ARG, "scale divisors give a singular V (repeated scales?)");
  for (int j = 0; j < N; ++j) {
    double Vj[49];
    std::memcpy(Vj, V, sizeof(double) * N * N);
    for (int row = 0; row < N; ++row) Vj[row * N + j] = d[row];
    c[j] = det_leibniz(Vj, N) / detV;
  }
  return YY_OK;
}

yy_status timing_begin(yy_ctx ctx) {
  if (!ctx->timing) return YY_OK;
  if (ctx->ev_used == ctx->ev_start.size()) {
    hipEvent_t a, b;
    YY_HIP(hipEventCreate(&a));
    YY_HIP(hipEventCreate(&b));
    ctx->ev_start.push_back(a);
    ctx->ev_stop.push_back(b);
  }
  YY_HIP(hipEventRecord(ctx->ev_start[ctx->ev_used], ctx->stream));
  return YY_OK;
}

yy_status timing_end(yy_ctx ctx) {
  if (!ctx->timing) return YY_OK;
  YY_HIP(hipEventRecord(ctx->ev_stop[ctx->ev_used], ctx->stream));
  ++ctx->ev_used;
  return YY_OK;
}

}  // namespace yy

using namespace yy;

extern "C" {

const char* yy_last_error(void) { return g_last_error.c_str(); }

yy_status yy_create(yy_ctx* out, int device, void* stream) {
  if (!out) return fail(YY_ERR_ARG, "yy_create: out is NULL");
  *out = nullptr;
  int count = 0;
  YY_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(YY_ERR_ARG, "yy_create: no such device");
  YY_HIP(hipSetDevice(device));
  {
    yy_status st = noalloc_scratch_init(device);
    if (st != YY_OK) return st;
  }
  yy_ctx ctx = new (std::nothrow) yy_ctx_s();
  if (!ctx) return fail(YY_ERR_ALLOC, "yy_create: out of host memory");
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipMalloc(&ctx->d_flags, 64);
  if (e != hipSuccess) {
    delete ctx;
    return hip_fail(e, "hipMalloc(status)");
  }
  ctx->d_nclamped = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(ctx->d_flags) + 8);
  ctx->d_defer = reinterpret_cast<int*>(reinterpret_cast<char*>(ctx->d_flags) + 16);
  e = hipMemsetAsync(ctx->d_flags, 0, 64, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(ctx->d_flags);
    delete ctx;
    return hip_fail(e, "hipMemsetAsync(status)");
  }
  *out = ctx;
  return YY_OK;
}

yy_status yy_destroy(yy_ctx ctx) {
  if (!ctx) return YY_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  ctx->d_dirs.release();
  ctx->prep.xc32.release();
  ctx->prep.f32.release();
  ctx->prep.bf.release();
  ctx->prep.f32t.release();
  ctx->bsrc.release();
  ctx->sflags.release();
  ctx->prep.node.release();
  ctx->prep.bnd.release();
  ctx->prep.scal.release();
  ctx->prep.div.release();
  ctx->prep.wtmp.release();
  ctx->prep.wnodes.release();
  ctx->prep.wbnd.release();
  ctx->obsw.release();
  ctx->rref.release();
  ctx->sym_items.release();
  ctx->tT.release();
  ctx->sym_list.release();
  ctx->fstar.release();
  ctx->lw2.release();
  ctx->part.release();
  ctx->red.release();
  ctx->red2.release();
  ctx->scan.release();
  for (hipEvent_t e : ctx->ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->ev_stop) (void)hipEventDestroy(e);
  (void)hipFree(ctx->d_flags);
  delete ctx;
  return YY_OK;
}

yy_status yy_set_stream(yy_ctx ctx, void* stream) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_set_stream: ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(stream);
  return YY_OK;
}

yy_status yy_get_status(yy_ctx ctx, uint32_t* flags, int64_t* nclamped) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_get_status: ctx is NULL");
  YY_HIP(hipSetDevice(ctx->device));
  uint64_t host[2] = {0, 0};
  YY_HIP(hipMemcpyAsync(host, ctx->d_flags, 16, hipMemcpyDeviceToHost, ctx->stream));
  YY_HIP(hipStreamSynchronize(ctx->stream));
  YY_HIP(hipMemsetAsync(ctx->d_flags, 0, 16, ctx->stream));
  YY_HIP(hipStreamSynchronize(ctx->stream));
  if (flags) *flags = (uint32_t)(host[0] & 0xFFFFFFFFu);
  if (nclamped) *nclamped = (int64_t)host[1];
  return YY_OK;
}

yy_status yy_timing_enable(yy_ctx ctx, int32_t on) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_timing_enable: ctx is NULL");
  ctx->timing = on != 0;
  return YY_OK;
}

yy_status yy_timing_read(yy_ctx ctx, double* ms, int64_t* launches) {
  if (!ctx) return fail(YY_ERR_ARG, "yy_timing_read: ctx is NULL");
  YY_HIP(hipSetDevice(ctx->device));
  YY_HIP(hipStreamSynchronize(ctx->stream));
  double total = 0.0;
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    float t = 0.f;
    YY_HIP(hipEventElapsedTime(&t, ctx->ev_start[i], ctx->ev_stop[i]));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = (int64_t)ctx->ev_used;
  ctx->ev_used = 0;
  return YY_OK;
}

yy_status yy_kernel_coefficients(int32_t S, const double* s, double* c_out) {
  if (S < 1 || S > YY_MAX_SCALES) return fail(YY_ERR_ARG, "yy_kernel_coefficients: S out of range");
  if (!s || !c_out) return fail(YY_ERR_ARG, "yy_kernel_coefficients: NULL pointer");
  for (int j = 0; j < S; ++j)
    if (!(s[j] > 0.0) || !std::isfinite(s[j])) return fail(YY_ERR_ARG, "scale divisors must be positive");
  return coefficients_cramer(S, s, c_out);
}

}  // extern "C"
