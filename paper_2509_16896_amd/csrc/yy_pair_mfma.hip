// yy_pair_mfma.hip -- the pairwise kernel on the CDNA4 matrix cores.
//
// For targets i and sources j (the same node set, centred at the box centre):
//   |x_i - x_j - tau_s f_j|^2 = |x_i|^2 + |m_j^s|^2 - 2 (G_ij + tau_s H_ij),
//   G = X X^T,  H = X F^T,  m_j^s = x_j + tau_s f_j,
// so one pass of two matrix products serves every scale s.  Each block owns
// 256 targets and a range of sources; per 128-source tile it accumulates G and
// H over K = r (zero padded to a multiple of 32 or 64) with MFMA 32x32 instructions
// (sources on the A side, targets on the B side, so every lane ends with one
// target and 16 sources per 32x32 block), then turns them into base-2
// exponents e = a_i + b_j + 2 kap_s G + 2 kap_s tau_s H and folds them into a
// running (max, sum) per (target, scale) held in the lane.
//
// Near pairs: every exponent within a rigorous error margin of the running
// maximum is recomputed exactly (FP32 direct differences, the self pair from
// the FP64 norm |f_i|^2), with the same arithmetic as the vector-ALU kernel,
// so the approximate products only ever contribute terms that are at least
// 2^-80 below the maximum.  Variants:
//   BF16X3:  hi/lo split of both operands, hi*hi + lo*hi + hi*lo, for G and H,
//   BF16X3G: the split for G only; H, which enters scaled by tau_s, is hi*hi,
//   BF16X1:  hi*hi only (a screen),  FP32: v_mfma_f32_32x32x2_f32 on FP32 data,
//   BF16X3S: a screen on G alone (k_pair_screen: H bounded, not computed) flags
//            the tiles that may hold a pair within 2^-80 of a row maximum;
//            BF16X3G then runs over the flagged tiles only,
//   BF16X3P: the same with a screen on the first 64 coordinates only
//            (k_pair_prescreen), whose partial squared distance bounds the
//            full one from below.
// Pull form (eq. kernel): the kernel is centred, as a function of the source,
// at x_i - tau_s f_i, so |x_i - tau_s f_i - x_j|^2 = |p_i^s|^2 + |x_j|^2
// - 2 (G_ij - tau_s H'_ij) with H' = F X^T: the targets carry the x and f
// planes, the sources only x, the target bias holds |p_i^s|^2 and the source
// bias |x_j|^2 (the factor exp(-tau_s div f(x_i)) enters in the combination).
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kMI = 256;   // targets per block
constexpr int kMJ = 128;   // sources per tile
constexpr int kKC = 16;    // K per LDS stage
#ifndef YY_PAIR_WAVES
#define YY_PAIR_WAVES 8
#endif
// Waves per block: 8 (2 per SIMD, 64 x 64 per wave) or 4 (1 per SIMD with the
// whole register file, 64 targets x 128 sources per wave).
constexpr int kWaves = YY_PAIR_WAVES;
static_assert(kWaves == 8 || kWaves == 4, "8 or 4 waves per block");
constexpr int kNT = 64 * kWaves;
constexpr int kWI = 4;                     // waves along targets
constexpr int kWJ = kWaves / kWI;          // waves along sources
constexpr int kIB = kMI / (32 * kWI);      // 32-wide target blocks per wave (64 targets)
constexpr int kJB = kMJ / (32 * kWJ);      // 32-wide source blocks per wave
constexpr float kSkip = 64.f;     // depth (bits) below the running maximum at which terms are dropped

struct MArgs {
  int64_t n, n_pad;
  int32_t r, rp, S;
  float kap[YY_MAX_SCALES];    // log2(e) s / (2 q dt)
  float c1[YY_MAX_SCALES];     // 2 kap_s
  float c2[YY_MAX_SCALES];     // 2 kap_s tau_s
  float tau[YY_MAX_SCALES];
  double kapd[YY_MAX_SCALES];
  double taud[YY_MAX_SCALES];
  const uint16_t* bf;          // bf16 planes [4][rp/16][n_pad][16]: hi(x), hi(f), lo(x), lo(f)
  const float* f32t;           // fp32 planes [2][rp/16][n_pad][16]: x, f
  const float* xc;             // row-major FP32 [n][rp] (exact near pairs)
  const float* f;
  const float* lw2;            // [n]
  const float* bsrc;           // [S][n_pad]: lw2_j - kap_s |m_j^s|^2, -inf for invalid sources
  const float* bpre;           // the same over the first kPreK coordinates (BF16X3P), or null
  const double* node;          // [6][n]: |x|^2, |f|^2, x.f, then the same over the first kPreK coordinates
  const double* scal;          // [1] = max |x - centre|, [2] = max |f|, [4], [5]: the same over kPreK
  const int* bnd;              // [n] boundary flags
  double eps_g, eps_h;         // relative error of one G / H product from operand rounding
  double eps_g1;               // the same for G in the screen of the screened split form
  float2* part;                // [nsplit][S][n]
  int32_t nsplit, tb_count, group_t;
  int64_t j_per_split;
  uint8_t* flags;              // screen verdicts [tb_count][jtl][8]: byte w < 4 for targets 64w..64w+63, 4..7 zero
  int64_t jtl;                 // source tiles of 128
  int32_t s_nsplit;            // the screen's source splits (of s_jps sources, a multiple of 256)
  int64_t s_jps;
  int32_t pre_chunks;          // 16-wide K stages of the partial-distance screen
  int* any_flag;               // deferred planes: k_src_bias clears it, the screen sets it on a flagged tile
  int32_t pull;                // pull-form kernel (biases and the sign of c2 follow it)
  const float* rref;           // [S][n] lower bounds of the row maxima (>= the self-pair exponent), or null
  const float* rhv;            // [S][n] with rref: the exact term of the pair (i, j*) where the row counts it
                               // at initialisation and leaves it out of the tiles, else -inf
  const long long* jstar;      // with rref: j*, the heaviest source (-1: none)
  // the symmetric partial-distance screen (BF16X3P on one run, many target blocks): its work items
  // (A, B0, B1): target block A against target blocks [B0, B1) as sources, B0 >= A; and per 64-row
  // group g and scale s the largest a_j^p + hx_j^p F^p - M_j over the group's valid rows with the
  // heavy pair counted apart (tT[s][g]) and without (tT[(S + s)][g])
  const int4* sym_items;
  const float* tT;
  int32_t sym_nitems, ngroups;
  // the units (B, group of 64 rows of B, A, wave of A) whose coarse bound doubted, for k_sym_recheck: a
  // counter (cleared by k_tgt_bound) and room for sym_cap entries
  int* sym_n;
  int4* sym_list;
  int32_t sym_cap;
};

// j* of the call (-1: none, or no rows floor), read once per block and kept in scalar registers
// (the argument set may come from global memory).
__device__ inline int64_t heavy_source(const MArgs& a) {
  const long long v = a.jstar ? *a.jstar : -1;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(unsigned long long)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Slab index jb * 16 + v, in the lane half g, of source offset d from the lane
// group's first source (the 32 x 32 accumulator layout: source 8 (v >> 2) +
// 4 g + (v & 3) of block jb); -1 if this lane half does not hold it.
template <int NJB>
__device__ inline int slab_index(int64_t d, int g) {
  return (d >= 0 && d < 32 * NJB && (int)((d >> 2) & 1) == g) ? (int)((d >> 5) * 16 + ((d >> 3) & 3) * 4 + (d & 3))
                                                               : -1;
}

// Physical 16-byte chunk of logical chunk c in LDS row `row` (bank-conflict swizzle).
// A 32-lane group reads 16 bytes from each of 32 consecutive rows; the XOR
// makes any 8 (16) consecutive rows hit distinct 16-byte slots of a 128-byte
// (256-byte) bank window.
template <int CPR>
__device__ inline int swz(int row, int c) {
  return CPR == 2 ? (c ^ ((row >> 2) & 1) ^ ((row >> 3) & 1)) : (c ^ ((row >> 1) & 3) ^ ((row >> 3) & 1));
}

// Block -> (target block, source split).  Blocks are dealt round-robin to the 8
// XCDs; each XCD walks a contiguous band of target blocks, `group_t` of them at
// a time with all their source splits, so a group's targets stay in that XCD's
// L2 while its source tiles are shared by `group_t` blocks.
__device__ inline void block_map(const MArgs& a, int& tb, int& split) {
  const int b = blockIdx.x;
  const int per_xcd = a.tb_count / 8;
  if (a.group_t > 0 && per_xcd > 0 && per_xcd * 8 == a.tb_count && per_xcd % a.group_t == 0) {
    const int xcd = b % 8, slot = b / 8;
    const int gsz = a.group_t * a.nsplit;
    const int grp = slot / gsz, rem = slot % gsz;
    tb = xcd * per_xcd + grp * a.group_t + rem % a.group_t;
    split = rem / a.group_t;
  } else {
    tb = b / a.nsplit;
    split = b % a.nsplit;
  }
}

// Parameters of the rare exact path, copied to LDS once per block so that the
// hot loop does not hold them in scalar registers.
struct Rare {
  const float* xc;
  const float* f;
  const float* lw2;
  const double* node;
  int64_t n;
  int32_t rp, pad;
  float kap[YY_MAX_SCALES], tau[YY_MAX_SCALES];
  double kapd[YY_MAX_SCALES], taud[YY_MAX_SCALES];
};

__device__ inline void fill_rare(const MArgs& a, Rare& rr) {
  rr.xc = a.xc;
  rr.f = a.f;
  rr.lw2 = a.lw2;
  rr.node = a.node;
  rr.n = a.n;
  rr.rp = a.rp;
  for (int s = 0; s < YY_MAX_SCALES; ++s) {
    rr.kap[s] = a.kap[s];
    rr.tau[s] = a.tau[s];
    rr.kapd[s] = a.kapd[s];
    rr.taud[s] = a.taud[s];
  }
}

// Exact base-2 exponent of a pair j != i by FP32 direct differences, summed in
// k order (zero-padded K adds exact zeros), the vector-ALU kernel's arithmetic:
// x_i - x_j - tau f_j (push form) or x_i - x_j - tau f_i (pull form).
template <bool PULL>
__device__ inline float exact_pair(const Rare& a, int64_t i, int64_t j, int s) {
  const float4* xi = reinterpret_cast<const float4*>(a.xc + (size_t)i * a.rp);
  const float4* xj = reinterpret_cast<const float4*>(a.xc + (size_t)j * a.rp);
  const float4* fj = reinterpret_cast<const float4*>(a.f + (size_t)(PULL ? i : j) * a.rp);
  const float t = a.tau[s];
  float acc = 0.f;
  const int nq = a.rp >> 2;
#pragma unroll 4
  for (int q = 0; q < nq; ++q) {
    const float4 p = xi[q], u = xj[q], w = fj[q];
    float e = fmaf(-t, w.x, p.x - u.x);
    acc = fmaf(e, e, acc);
    e = fmaf(-t, w.y, p.y - u.y);
    acc = fmaf(e, e, acc);
    e = fmaf(-t, w.z, p.z - u.z);
    acc = fmaf(e, e, acc);
    e = fmaf(-t, w.w, p.w - u.w);
    acc = fmaf(e, e, acc);
  }
  return a.lw2[j] - a.kap[s] * acc;
}

// Folds the accumulators of one target (kJB blocks x 16 sources of this lane)
// into the lane's running (max, sum) of that target for every scale.
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ inline void lse2_push(float& M, float& S, float v) {
  if (v == -INFINITY) return;
  if (v > M) {
    S = S * fast_exp2(M - v) + 1.f;
    M = v;
  } else {
    S += fast_exp2(v - M);
  }
}

// The rare path of a slab that reaches within 2^-64 of the running maximum:
// exponents within `margin` of the maximum are recomputed exactly, the others
// are summed from their approximate values.  Out of line so that the hot
// loop's register allocation does not carry it.  e: the 16 kJB approximate
// exponents (self pair already -inf); returns the new (max, sum).
constexpr int kSlab = 16 * kJB;
template <bool PULL>
__device__ __noinline__ float2 refine_slab(const Rare* rr, int64_t i, int64_t jbase, int g, int s,
                                           float margin, const float* e, float M, float S) {
  float m = -INFINITY;
  for (int b = 0; b < kSlab; ++b) m = fmaxf(m, e[b]);
  const float thr = fmaxf(M, m) - margin;
  float m2 = -INFINITY;
  for (int b = 0; b < kSlab; ++b) {
    if (e[b] >= thr) {
      const int jb = b >> 4, v = b & 15;
      const int64_t j = jbase + jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
      lse2_push(M, S, exact_pair<PULL>(*rr, i, j, s));
    } else {
      m2 = fmaxf(m2, e[b]);
    }
  }
  const float Mn = fmaxf(M, m2);
  if (Mn == -INFINITY) return make_float2(M, S);
  float sum = S * fast_exp2(M - Mn);
  for (int b = 0; b < kSlab; ++b)
    if (e[b] < thr) sum += fast_exp2(e[b] - Mn);
  return make_float2(Mn, sum);
}

template <int S, bool PULL>
__device__ inline void epilogue_target(const MArgs& a, const Rare* rare, const f32x16_t (&G)[kJB],
                                       const f32x16_t (&H)[kJB], const float* sb, int64_t i, int64_t j0,
                                       int jl0, int g, bool diag, int bheavy, const float (&at)[S],
                                       const float (&margin)[S], float (&M)[S], float (&Ssum)[S]) {
  // The self pair (source j = i) is accounted for at initialisation; this
  // lane holds it iff d = i - j0 - jl0 is in [0, 32 kJB) with bit 2 equal to g.
  // bself: its slab index in this lane (-1: none); bheavy: the same for the
  // pair (i, j*) where the row counts that one at initialisation too.
  const int bself = diag ? slab_index<kJB>(i - j0 - jl0, g) : -1;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float c1 = a.c1[s], c2 = a.c2[s];
    float m = -INFINITY;
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int jl = jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
        float e = fmaf(c2, H[jb][v], fmaf(c1, G[jb][v], at[s] + sb[s * kMJ + jl0 + jl]));
        if (jb * 16 + v == bself || jb * 16 + v == bheavy) e = -INFINITY;
        m = fmaxf(m, e);
      }
    // Every exact exponent of the slab is at most m + (margin - kSkip - 16): below
    // 2^-(kSkip+16) of the running maximum unless m > M - margin.
    if (!(m > M[s] - margin[s])) continue;
    float e[kSlab];
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int jl = jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
        float x = fmaf(c2, H[jb][v], fmaf(c1, G[jb][v], at[s] + sb[s * kMJ + jl0 + jl]));
        if (jb * 16 + v == bself || jb * 16 + v == bheavy) x = -INFINITY;
        e[jb * 16 + v] = x;
      }
    const float2 r = refine_slab<PULL>(rare, i, j0 + jl0, g, s, margin[s], e, M[s], Ssum[s]);
    M[s] = r.x;
    Ssum[s] = r.y;
  }
}

// Final merge: lanes l and l^32 hold the same target; with two waves along
// the sources, waves (wi, 0) and (wi, 1) hold the same targets.  Writes
// part[split][s][i].
template <int S>
__device__ inline void merge_and_store(const MArgs& a, float (&M)[kIB][S], float (&Ssum)[kIB][S],
                                       int64_t i0, int split, float2* xchg) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float mo = __shfl_xor(M[ib][s], 32, 64);
      const float so = __shfl_xor(Ssum[ib][s], 32, 64);
      lse2_merge(M[ib][s], Ssum[ib][s], mo, so);
    }
  if (kWJ == 2) {
    __syncthreads();
    if (wj == 1 && g == 0) {
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int s = 0; s < S; ++s)
          xchg[((wi * kIB + ib) * 32 + col) * S + s] = make_float2(M[ib][s], Ssum[ib][s]);
    }
    __syncthreads();
  }
  if (wj == 0 && g == 0) {
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (kWJ == 2) {
          const float2 o = xchg[((wi * kIB + ib) * 32 + col) * S + s];
          lse2_merge(M[ib][s], Ssum[ib][s], o.x, o.y);
        }
        if (i < a.n) a.part[((size_t)split * S + s) * a.n + i] = make_float2(M[ib][s], Ssum[ib][s]);
      }
    }
  }
}

// Rigorous bound on |e_approx - e_exact| in base-2 units: operand rounding,
// worst-case FP32 accumulation over rp products, FP32 evaluation of e; the
// margin adds the skip depth and 16 bits of safety.
template <int S>
__device__ inline void init_targets(const MArgs& a, int64_t i0, int split, float (&at)[kIB][S],
                                    float (&M)[kIB][S], float (&Ssum)[kIB][S], float (&margin)[S],
                                    bool (&hv)[kIB]) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
  const double X = a.scal[1], F = a.scal[2];
  const double gam = a.rp * 0x1p-24;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double XT = X + a.taud[s] * F;
    const double dD = 2.0 * X * ((a.eps_g + gam) * X + (a.eps_h + gam) * a.taud[s] * F) + 16.0 * 0x1p-24 * XT * XT;
    margin[s] = (float)(2.0 * a.kapd[s] * dD + (double)kSkip + 16.0);
  }
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
    const bool valid = i < a.n;
    const double nx = valid ? a.node[i] : 0.0;
    const double nf = valid ? a.node[a.n + i] : 0.0;
    const double nxf = valid ? a.node[2 * a.n + i] : 0.0;
    const float li = valid ? a.lw2[i] : -INFINITY;
    // The self pair is one of the terms, so its exact exponent bounds the row
    // maximum from below: every partial state starts at it (tiles far below
    // are then skipped untouched) and exactly one state -- the one whose
    // source range holds j = i -- starts with it counted.  Where the row's
    // bound is the pair with the heaviest source j*, that state also counts
    // that pair's exact term, and the tiles leave it out (hv).
    const bool owner = valid && (int64_t)split == i / a.j_per_split && wj == (int)((i % kMJ) / (32 * kJB)) &&
                       g == (int)((i >> 2) & 1);
    hv[ib] = valid && a.rhv && a.rhv[i] != -INFINITY;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // target term: -kap |x_i|^2 (push), -kap |x_i - tau f_i|^2 (pull)
      const double t = a.taud[s];
      at[ib][s] = valid ? (float)(-a.kapd[s] * (a.pull ? nx - 2.0 * t * nxf + t * t * nf : nx)) : -INFINITY;
      // the running maximum starts at the row's lower bound (the self pair, or the exact term of
      // the heaviest source where that is larger); the owner counts the self term relative to it
      const float self = (valid && li != -INFINITY) ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf) : -INFINITY;
      const float ref = (valid && a.rref) ? a.rref[(size_t)s * a.n + i] : self;
      M[ib][s] = ref;
      Ssum[ib][s] = (owner && self != -INFINITY) ? (self == ref ? 1.f : fast_exp2(self - ref)) : 0.f;
      if (owner && hv[ib]) {
        const float h = a.rhv[(size_t)s * a.n + i];
        Ssum[ib][s] += h == ref ? 1.f : fast_exp2(h - ref);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Global -> LDS pipeline.  Every 1 KB region of a stage is filled by one
// global_load_lds_dwordx4 of one wave (lane L's 16 bytes land at byte 16 L of
// the region), so the bank-conflict swizzle is applied by choosing which
// global chunk a lane fetches.  The copies are issued through inline asm: the
// compiler then neither inserts conservative vmcnt waits before unrelated LDS
// reads nor keeps LDS values in registers across them ("memory" clobber); the
// kernel waits for each stage explicitly with s_waitcnt vmcnt before the
// barrier that publishes it.  M0 is saved and restored around the copy.
__device__ inline uint32_t lds_addr(const void* p) {
  return (uint32_t)reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) void*)p);
}

__device__ inline void dma_1k(const void* gsrc, uint32_t lds) {
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds), "v"(gsrc)
      : "memory");
}

// s_waitcnt immediate that waits until at most V vector-memory operations of
// this wave are outstanding (expcnt and lgkmcnt left unconstrained).
template <int V>
__device__ inline void wait_vmcnt() {
  static_assert(V >= 0 && V < 64, "vmcnt out of range");
  __builtin_amdgcn_s_waitcnt((V & 15) | ((V >> 4) << 14) | 0x70 | 0xF00);
}

// Issues the copies of one K stage: target planes (rows i0..i0+255) then source
// planes (rows j0..j0+127) of K chunk c.  ESZ = element bytes (2: bf16, 4: fp32).
// Global planes are [chunk][n_pad][16 elements] (hi(x), hi(f), lo(x), lo(f));
// push form: target planes are global planes 0 and 2, source planes 0..3; pull
// form the other way round.
template <int ESZ, int NTP, int NSP, bool PULL = false>
__device__ inline void issue_stage(const unsigned char* gb, uint64_t plane_bytes, int64_t n_pad,
                                   uint32_t stage_lds, int c, int64_t i0, int64_t j0, int wave, int lane) {
  constexpr int ROWB = kKC * ESZ;              // bytes per row per stage
  constexpr int CPR = ROWB / 16;               // 16-byte chunks per row
  constexpr int RPR = 64 / CPR;                // rows per 1 KB region
  constexpr int TREG = kMI / RPR, SREG = kMJ / RPR;
  constexpr int R = NTP * TREG + NSP * SREG;
  constexpr int RW = (R + kWaves - 1) / kWaves;
  const unsigned char* tb = gb + ((uint64_t)c * (uint64_t)n_pad + (uint64_t)i0) * ROWB;
  const unsigned char* sbp = gb + ((uint64_t)c * (uint64_t)n_pad + (uint64_t)j0) * ROWB;
  const int rl = lane / CPR, pc = lane % CPR;
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    const int q = wave + kWaves * u;   // wave-uniform
    if (R % kWaves != 0 && q >= R) break;
    const unsigned char* src;
    int off;
    if (q < NTP * TREG) {
      const int p = q / TREG, rb = (q % TREG) * RPR, row = rb + rl;
      src = tb + (uint64_t)(PULL ? p : 2 * p) * plane_bytes + row * ROWB + swz<CPR>(row, pc) * 16;
      off = p * (kMI * ROWB) + rb * ROWB;
    } else {
      const int q2 = q - NTP * TREG;
      const int p = q2 / SREG, rb = (q2 % SREG) * RPR, row = rb + rl;
      src = sbp + (uint64_t)(PULL ? 2 * p : p) * plane_bytes + row * ROWB + swz<CPR>(row, pc) * 16;
      off = NTP * kMI * ROWB + p * (kMJ * ROWB) + rb * ROWB;
    }
    dma_1k(src, stage_lds + off);
  }
}

// The lane index, recomputed where it is used: the compiler may neither merge
// nor hoist the asm statement, so addresses derived from it are not kept live
// (or spilled) across the main loop; a spill reload would wait for every copy
// in flight, since it shares their vmcnt counter.
__device__ inline int fresh_lane() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// Source biases of tile j0 -> sb (wave 0 only): [S][128] floats, lane-ordered.
__device__ inline void issue_bias(const MArgs& a, uint32_t sb_lds, int64_t j0, int wave) {
  if (wave != 0) return;
  const int lane = fresh_lane();
  const int regions = (a.S * kMJ * 4 + 1023) / 1024;
  for (int u = 0; u < regions; ++u) {
    const int idx = 256 * u + 4 * lane;
    int s = idx / kMJ;
    if (s >= a.S) s = a.S - 1;   // lanes past the last scale fetch a valid address; never read
    const float* src = a.bsrc + (size_t)s * a.n_pad + j0 + (idx % kMJ);
    dma_1k(src, sb_lds + u * 1024);
  }
}

template <int S>
__device__ inline void zero_acc(f32x16_t (&G)[kIB][kJB], f32x16_t (&H)[kIB][kJB]) {
#pragma unroll
  for (int x = 0; x < kIB; ++x)
#pragma unroll
    for (int y = 0; y < kJB; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        G[x][y][v] = 0.f;
        H[x][y][v] = 0.f;
      }
}

// One K stage of the products on the matrix cores, in two halves: the
// fragment reads from LDS (into a Frag) and the matrix-core burst, so that the
// reads of the next stage can be issued ahead of the current burst.  PASSES:
// 3 = split G and H, 2 = split G with H hi*hi, 1 = hi*hi only.
struct Frag {
  bf16x8_t bh[kIB], bl[kIB], xh[kJB], xl[kJB], fh[kJB], fl[kJB];
};

template <int PASSES>
__device__ inline void load_frags(const unsigned char* base, Frag& f) {
  constexpr int ROWB = 32;
  constexpr int NTP = PASSES >= 2 ? 2 : 1;
  constexpr int TB = NTP * kMI * ROWB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
  bf16x8_t(&bh)[kIB] = f.bh;
  bf16x8_t(&bl)[kIB] = f.bl;
  bf16x8_t(&xh)[kJB] = f.xh;
  bf16x8_t(&xl)[kJB] = f.xl;
  bf16x8_t(&fh)[kJB] = f.fh;
  bf16x8_t(&fl)[kJB] = f.fl;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int row = wi * (32 * kIB) + ib * 32 + col;
    const int off = row * ROWB + swz<2>(row, g) * 16;
    bh[ib] = *reinterpret_cast<const bf16x8_t*>(base + off);
    if (PASSES >= 2) bl[ib] = *reinterpret_cast<const bf16x8_t*>(base + kMI * ROWB + off);
  }
#pragma unroll
  for (int jb = 0; jb < kJB; ++jb) {
    const int row = wj * (32 * kJB) + jb * 32 + col;
    const int off = TB + row * ROWB + swz<2>(row, g) * 16;
    xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + off);
    fh[jb] = *reinterpret_cast<const bf16x8_t*>(base + kMJ * ROWB + off);
    if (PASSES >= 2) xl[jb] = *reinterpret_cast<const bf16x8_t*>(base + 2 * kMJ * ROWB + off);
    if (PASSES == 3) fl[jb] = *reinterpret_cast<const bf16x8_t*>(base + 3 * kMJ * ROWB + off);
  }
}

template <int PASSES>
__device__ inline void mma_frags(const Frag& f, f32x16_t (&G)[kIB][kJB], f32x16_t (&H)[kIB][kJB]) {
  const bf16x8_t(&bh)[kIB] = f.bh;
  const bf16x8_t(&bl)[kIB] = f.bl;
  const bf16x8_t(&xh)[kJB] = f.xh;
  const bf16x8_t(&xl)[kJB] = f.xl;
  const bf16x8_t(&fh)[kJB] = f.fh;
  const bf16x8_t(&fl)[kJB] = f.fl;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb) {
      G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bh[ib], G[ib][jb], 0, 0, 0);
      H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[jb], bh[ib], H[ib][jb], 0, 0, 0);
      if (PASSES >= 2) {
        G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[jb], bh[ib], G[ib][jb], 0, 0, 0);
        G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bl[ib], G[ib][jb], 0, 0, 0);
      }
      if (PASSES == 3) {
        H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl[jb], bh[ib], H[ib][jb], 0, 0, 0);
        H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[jb], bl[ib], H[ib][jb], 0, 0, 0);
      }
    }
}

// Pull form: the target side carries hi(x), hi(f), lo(x), lo(f) (as many as
// the variant needs, in that order), the source side hi(x), lo(x).
struct FragP {
  bf16x8_t bh[kIB], bfh[kIB], bl[kIB], bfl[kIB], xh[kJB], xl[kJB];
};

template <int PASSES>
__device__ inline void load_frags_pull(const unsigned char* base, FragP& f) {
  constexpr int ROWB = 32;
  constexpr int NTP = PASSES == 3 ? 4 : PASSES == 2 ? 3 : 2;
  constexpr int TB = NTP * kMI * ROWB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int row = wi * (32 * kIB) + ib * 32 + col;
    const int off = row * ROWB + swz<2>(row, g) * 16;
    f.bh[ib] = *reinterpret_cast<const bf16x8_t*>(base + off);
    f.bfh[ib] = *reinterpret_cast<const bf16x8_t*>(base + kMI * ROWB + off);
    if (PASSES >= 2) f.bl[ib] = *reinterpret_cast<const bf16x8_t*>(base + 2 * kMI * ROWB + off);
    if (PASSES == 3) f.bfl[ib] = *reinterpret_cast<const bf16x8_t*>(base + 3 * kMI * ROWB + off);
  }
#pragma unroll
  for (int jb = 0; jb < kJB; ++jb) {
    const int row = wj * (32 * kJB) + jb * 32 + col;
    const int off = TB + row * ROWB + swz<2>(row, g) * 16;
    f.xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + off);
    if (PASSES >= 2) f.xl[jb] = *reinterpret_cast<const bf16x8_t*>(base + kMJ * ROWB + off);
  }
}

// G = X X^T as in the push form; H'_ij = x_j . f_i (sources x on the A side, target f on the B side)
template <int PASSES>
__device__ inline void mma_frags_pull(const FragP& f, f32x16_t (&G)[kIB][kJB], f32x16_t (&H)[kIB][kJB]) {
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb) {
      G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[jb], f.bh[ib], G[ib][jb], 0, 0, 0);
      H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[jb], f.bfh[ib], H[ib][jb], 0, 0, 0);
      if (PASSES >= 2) {
        G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xl[jb], f.bh[ib], G[ib][jb], 0, 0, 0);
        G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[jb], f.bl[ib], G[ib][jb], 0, 0, 0);
      }
      if (PASSES == 3) {
        H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xl[jb], f.bfh[ib], H[ib][jb], 0, 0, 0);
        H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[jb], f.bfl[ib], H[ib][jb], 0, 0, 0);
      }
    }
}

// FP32: within a 16-wide K stage, lane group g owns k = 8 g + t in K step t
// (any fixed assignment of k to steps is valid when both operands use it), so
// a lane reads two consecutive 16-byte chunks of its row.
template <bool PULL = false>
__device__ inline void mfma_stage_f32(const unsigned char* base, f32x16_t (&G)[kIB][kJB],
                                      f32x16_t (&H)[kIB][kJB]) {
  constexpr int ROWB = 64;
  constexpr int TB = (PULL ? 2 : 1) * kMI * ROWB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int lc = 2 * g + u;
    float4 bt[kIB], bf[kIB], xs[kJB], fs[kJB];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int row = wi * (32 * kIB) + ib * 32 + col;
      const int off = row * ROWB + swz<4>(row, lc) * 16;
      bt[ib] = *reinterpret_cast<const float4*>(base + off);
      if (PULL) bf[ib] = *reinterpret_cast<const float4*>(base + kMI * ROWB + off);
    }
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb) {
      const int row = wj * (32 * kJB) + jb * 32 + col;
      const int off = TB + row * ROWB + swz<4>(row, lc) * 16;
      xs[jb] = *reinterpret_cast<const float4*>(base + off);
      if (!PULL) fs[jb] = *reinterpret_cast<const float4*>(base + kMJ * ROWB + off);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < kJB; ++jb) {
          G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[jb][e], bt[ib][e], G[ib][jb], 0, 0, 0);
          if (PULL)
            H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[jb][e], bf[ib][e], H[ib][jb], 0, 0, 0);
          else
            H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(fs[jb][e], bt[ib][e], H[ib][jb], 0, 0, 0);
        }
  }
}

// The pairwise kernel.  VAR: 3 = BF16 hi/lo split of G and H, 2 = split of G
// only, 1 = BF16 hi only, 0 = FP32.
// The (source tile, K chunk) steps of a block form one flat sequence, taken
// in groups of SPB steps, one barrier per group.  The LDS ring holds NS
// stages = NS / SPB groups: while one group is consumed the copies of the
// next LA = NS / SPB - 1 groups are in flight, so the pipeline keeps running
// across tile boundaries while a tile's epilogue folds its products into the
// running (max, sum).
template <int VAR, bool PULL = false>
struct StageShape {
  static constexpr int ESZ = VAR == 0 ? 4 : 2;                       // element bytes
  static constexpr int XP = VAR >= 2 ? 2 : 1;                        // planes of the side without f
  static constexpr int FP = VAR == 3 ? 4 : VAR == 2 ? 3 : 2;         // planes of the side with f
  static constexpr int NTP = PULL ? FP : XP;                         // target planes
  static constexpr int NSP = PULL ? XP : FP;                         // source planes
  static constexpr int ROWB = kKC * ESZ;
  static constexpr int STAGE = (NTP * kMI + NSP * kMJ) * ROWB;       // bytes per LDS stage
};

// One block's work: targets [256 tb, 256 tb + 256) against the sources of split
// `split`, partial (max, sum) to a.part.  smem, sbuf, rare and tl are the
// block's LDS ring, bias buffers, rare-path parameters and tile list.
// FLAGGED: only the tiles flagged by the screen (k_pair_screen below), taken
// in windows of kTileWindow tiles; the others hold no pair within 2^-80 of a
// row maximum.
constexpr int kTileWindow = 64;

template <int S, int VAR, int NS, int SPB, bool FLAGGED, bool PULL = false>
__device__ __forceinline__ void pair_block(const MArgs& a, int tb, int split, unsigned char* smem,
                                           float (*sbuf)[4 * kMJ], Rare& rare, int* tl) {
  static_assert(NS % SPB == 0 && NS / SPB >= 2, "the ring holds at least two groups of stages");
  static_assert(!(PULL && FLAGGED), "the screened forms are push-form only");
  constexpr int LA = NS / SPB - 1;
  constexpr int ESZ = StageShape<VAR, PULL>::ESZ;
  constexpr int NTP = StageShape<VAR, PULL>::NTP;
  constexpr int NSP = StageShape<VAR, PULL>::NSP;
  constexpr int STAGE = StageShape<VAR, PULL>::STAGE;
  constexpr int L = STAGE / 1024 / kWaves;     // copies per wave per stage
  static_assert(LA == 1 || L * kWaves * 1024 == STAGE, "deep lookahead needs equal copies per wave");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
  const int64_t i0 = (int64_t)tb * kMI;
  const int64_t jb0 = (int64_t)split * a.j_per_split;
  const int64_t jb1 = jb0 + a.j_per_split < a.n ? jb0 + a.j_per_split : a.n;
  // block-uniform counts (the LDS addresses of the copies derive from them and
  // must live in scalar registers even when `a` was read from global memory)
  const int ntiles_all = __builtin_amdgcn_readfirstlane((int)((jb1 - jb0 + kMJ - 1) / kMJ));
  const int nchunks = __builtin_amdgcn_readfirstlane(a.rp / kKC);
  const int64_t jt0 = jb0 / kMJ;   // global index of the split's first source tile
  // no tile flagged in this call: every split keeps its starting state, and the combination forms
  // the one of the split that holds each target's self pair itself (owner_start), reading no other
  if (FLAGGED && a.any_flag && *a.any_flag == 0) return;
  if (FLAGGED) {
    // A source range without a flagged tile leaves every partial state as it
    // starts (the self-pair exponent; sum 1 in the split that holds the self
    // pair, else 0): those are written directly, the value merge_and_store
    // would produce.
    if (wave == 0) {
      bool any = false;
      for (int w0 = 0; w0 < ntiles_all; w0 += 64)
        any |= w0 + lane < ntiles_all &&
               *reinterpret_cast<const uint64_t*>(a.flags + ((size_t)tb * a.jtl + jt0 + w0 + lane) * 8) != 0;
      any = __any(any);
      if (lane == 0) tl[kTileWindow] = any ? 1 : 0;
    }
    __syncthreads();
    if (tl[kTileWindow] == 0) {
      if (tid < kMI) {
        const int64_t i = i0 + tid;
        const bool own = (int64_t)split == i / a.j_per_split;
        if (i < a.n) {
          const float li = a.lw2[i];
          const double nf = a.node[a.n + i];
#pragma unroll
          for (int s = 0; s < S; ++s) {
            float2 v = owner_start(li, nf, a.kapd[s], a.taud[s], a.rref, a.rhv, a.n, i, s);
            if (!own) v.y = 0.f;
            a.part[((size_t)split * S + s) * a.n + i] = v;
          }
        }
      }
      return;
    }
  }
  if (tid == 0) fill_rare(a, rare);
  const uint64_t plane = (uint64_t)nchunks * a.n_pad * kKC * ESZ;   // bytes per global plane
  const unsigned char* gb = VAR == 0 ? reinterpret_cast<const unsigned char*>(a.f32t)
                                     : reinterpret_cast<const unsigned char*>(a.bf);
  const int64_t n_pad = a.n_pad;
  const uint32_t smem_lds = __builtin_amdgcn_readfirstlane(lds_addr(smem));
  const uint32_t sb_lds = __builtin_amdgcn_readfirstlane(lds_addr(&sbuf[0][0]));

  float at[kIB][S], M[kIB][S], Ssum[kIB][S], margin[S];
  bool hv[kIB];
  init_targets<S>(a, i0, split, at, M, Ssum, margin, hv);
  const int64_t jstar = heavy_source(a);

  for (int w0 = 0; w0 < ntiles_all; w0 += FLAGGED ? kTileWindow : ntiles_all) {
    int ntiles = ntiles_all;
    if (FLAGGED) {
      // the window's flagged tiles, in order
      const int wn = ntiles_all - w0 < kTileWindow ? ntiles_all - w0 : kTileWindow;
      __syncthreads();   // the previous window is done with the ring, the bias buffers and the list
      if (wave == 0) {
        const bool f = lane < wn &&
                       *reinterpret_cast<const uint64_t*>(a.flags + ((size_t)tb * a.jtl + jt0 + w0 + lane) * 8) != 0;
        const uint64_t mask = __ballot(f);
        if (f) tl[__popcll(mask & ((1ull << lane) - 1))] = w0 + lane;
        if (lane == 0) tl[kTileWindow] = __popcll(mask);
      }
      __syncthreads();
      ntiles = __builtin_amdgcn_readfirstlane(tl[kTileWindow]);
      if (ntiles == 0) continue;
    }
    // first source of the window's tile t
    auto tile_j0 = [&](int t) -> int64_t {
      return jb0 + (int64_t)(FLAGGED ? __builtin_amdgcn_readfirstlane(tl[t]) : t) * kMJ;
    };
    const int Q = ntiles * nchunks;

    issue_bias(a, sb_lds, tile_j0(0), wave);
#pragma unroll
    for (int p = 0; p < LA * SPB; ++p)
      if (p < Q) issue_stage<ESZ, NTP, NSP, PULL>(gb, plane, n_pad, smem_lds + p * STAGE, p % nchunks, i0,
                                                  tile_j0(p / nchunks), wave, lane);

    for (int t = 0; t < ntiles; ++t) {
      const int64_t j0 = tile_j0(t);
      f32x16_t G[kIB][kJB], H[kIB][kJB];
      zero_acc<S>(G, H);
      for (int c = 0; c < nchunks; c += SPB) {
        const int q = t * nchunks + c;
        // this wave's copies of steps q .. q+SPB-1 have landed (the later groups
        // may still fly, unless a tile has so few groups that the copies waited
        // for here were issued before the biases of the tile ending here) ...
        if (q + LA * SPB - 1 < Q && 2 * (nchunks / SPB) - 1 >= LA) wait_vmcnt<(LA - 1) * SPB * L>();
        else wait_vmcnt<0>();
        __syncthreads();   // ... for every wave; the previous group's stages are free again
        if (c == 0 && t + 1 < ntiles)
          issue_bias(a, sb_lds + ((t + 1) & 1) * (4 * kMJ * 4), tile_j0(t + 1), wave);
#pragma unroll
        for (int u = 0; u < SPB; ++u) {
          const int qn = q + LA * SPB + u;
          if (qn < Q) {
            const int tn = qn / nchunks;
            issue_stage<ESZ, NTP, NSP, PULL>(gb, plane, n_pad, smem_lds + (qn % NS) * STAGE, qn - tn * nchunks,
                                             i0, tile_j0(tn), wave, lane);
          }
        }
        if (VAR == 0) {
#pragma unroll
          for (int u = 0; u < SPB; ++u) mfma_stage_f32<PULL>(smem + ((q + u) % NS) * STAGE, G, H);
        } else if (PULL) {
          FragP fr[2];
          load_frags_pull<VAR>(smem + (q % NS) * STAGE, fr[0]);
#pragma unroll
          for (int u = 0; u < SPB; ++u) {
            if (u + 1 < SPB) load_frags_pull<VAR>(smem + ((q + u + 1) % NS) * STAGE, fr[(u + 1) & 1]);
            mma_frags_pull<VAR>(fr[u & 1], G, H);
          }
        } else {
          // fragments of stage u + 1 are read while the burst of stage u runs
          Frag fr[2];
          load_frags<VAR>(smem + (q % NS) * STAGE, fr[0]);
#pragma unroll
          for (int u = 0; u < SPB; ++u) {
            if (u + 1 < SPB) load_frags<VAR>(smem + ((q + u + 1) % NS) * STAGE, fr[(u + 1) & 1]);
            mma_frags<VAR>(fr[u & 1], G, H);
          }
        }
      }
      const float* sb = &sbuf[t & 1][0];
      const bool diag = j0 < i0 + kMI && i0 < j0 + kMJ;
      const bool htile = jstar >= j0 && jstar < j0 + kMJ;
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) {
        const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
        const int bheavy = (htile && hv[ib]) ? slab_index<kJB>(jstar - j0 - wj * (32 * kJB), g) : -1;
        // keep one target's accumulators in flight at a time (register pressure)
        __builtin_amdgcn_sched_barrier(0);
        epilogue_target<S, PULL>(a, &rare, G[ib], H[ib], sb, i, j0, wj * (32 * kJB), g, diag, bheavy, at[ib],
                                 margin, M[ib], Ssum[ib]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  merge_and_store<S>(a, M, Ssum, i0, split, reinterpret_cast<float2*>(smem));
}

template <int S, int VAR, int NS, int SPB, bool FLAGGED, bool PULL = false>
__global__ void __launch_bounds__(kNT, 1) k_pair_mfma(MArgs a) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * StageShape<VAR, PULL>::STAGE];
  __shared__ __attribute__((aligned(1024))) float sbuf[2][4 * kMJ];
  __shared__ Rare rare;
  __shared__ int tl[FLAGGED ? kTileWindow + 1 : 1];
  int tb, split;
  block_map(a, tb, split);
  pair_block<S, VAR, NS, SPB, FLAGGED, PULL>(a, tb, split, smem, sbuf, rare, tl);
}

// Many node sets in one launch: block b takes work item items[b] = (set,
// target block, source split); the items come in decreasing cost order.
template <int S, int VAR, int NS, int SPB, bool FLAGGED>
__global__ void __launch_bounds__(kNT, 1) k_pair_mfma_batch(const MArgs* __restrict__ sets,
                                                            const int4* __restrict__ items) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * StageShape<VAR>::STAGE];
  __shared__ __attribute__((aligned(1024))) float sbuf[2][4 * kMJ];
  __shared__ Rare rare;
  __shared__ int tl[FLAGGED ? kTileWindow + 1 : 1];
  const int4 it = items[blockIdx.x];
  pair_block<S, VAR, NS, SPB, FLAGGED>(sets[__builtin_amdgcn_readfirstlane(it.x)], __builtin_amdgcn_readfirstlane(it.y),
                                    __builtin_amdgcn_readfirstlane(it.z), smem, sbuf, rare, tl);
}

// ---------------------------------------------------------------------------
// The screen of the screened split form, on G = X X^T alone.  The tau-scaled
// term is bounded instead of computed: |2 kap_s tau_s x_i.f_j| <= hx_i F with
// hx_i = (log2 e / q) |x_i| (kap_s tau_s does not depend on s) and F = max_j
// |f_j| (Cauchy-Schwarz), so
//   e_exact <= a_i + hx_i F + b_js + 2 kap_s G~_ij + err_G,
// err_G the rigorous error of the one-product G (operand rounding, FP32
// accumulation and evaluation).  Without the H accumulators a wave holds 64
// targets x 128 sources, so a block tile is 256 x 256 and one 16-wide K stage
// (the hi planes of x only) is 16 KB: half the bytes and half the products per
// pair of a screen that also forms H.  A wave's 64 x 128 sub-tile is one
// 128-source tile of the split pass, whose flag byte the wave writes.
constexpr int kSJ = 256;                      // sources per screen tile
constexpr int kSJB = kSJ / (32 * kWJ);        // 32-wide source blocks per wave
constexpr int kSStage = (kMI + kSJ) * 32;     // bytes per LDS stage (hi(x) of targets and sources)
constexpr int kSBRows = 4;                    // bias rows per screen tile (up to 4 scales)
static_assert(kWaves == 8, "the screen tile assumes 8 waves");

struct SFrag {
  bf16x8_t bh[kIB], xh[kSJB];
};

__device__ inline void screen_load_frags(const unsigned char* base, SFrag& f, int wave) {
  constexpr int ROWB = 32;
  const int lane = fresh_lane();
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int row = wi * (32 * kIB) + ib * 32 + col;
    f.bh[ib] = *reinterpret_cast<const bf16x8_t*>(base + row * ROWB + swz<2>(row, g) * 16);
  }
#pragma unroll
  for (int jb = 0; jb < kSJB; ++jb) {
    const int row = wj * (32 * kSJB) + jb * 32 + col;
    f.xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + kMI * ROWB + row * ROWB + swz<2>(row, g) * 16);
  }
}

__device__ inline void screen_mma(const SFrag& f, f32x16_t (&G)[kIB][kSJB]) {
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
    for (int jb = 0; jb < kSJB; ++jb)
      G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[jb], f.bh[ib], G[ib][jb], 0, 0, 0);
}

// One screen stage: 8 target and 8 source regions of 1 KB (32 rows of hi(x)),
// two per wave.
__device__ inline void screen_issue_stage(const unsigned char* gb, int64_t n_pad, uint32_t stage_lds, int c,
                                          int64_t i0, int64_t j0, int wave) {
  constexpr int ROWB = 32;
  const int lane = fresh_lane(), rl = lane >> 1, pc = lane & 1;
  const int loff = rl * ROWB + swz<2>(rl, pc) * 16;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = wave + 8 * u;   // wave-uniform: 0..7 targets, 8..15 sources
    const int64_t row0 = (u == 0 ? i0 : j0) + (q & 7) * 32;
    dma_1k(gb + ((uint64_t)c * (uint64_t)n_pad + (uint64_t)row0) * ROWB + loff, stage_lds + q * 1024);
  }
}

// Source biases bs of the S scales of screen tile j0 (wave 0): [S][256] floats.
__device__ inline void screen_issue_bias(const MArgs& a, const float* bs, uint32_t sb_lds, int64_t j0, int wave) {
  if (wave != 0) return;
  const int lane = fresh_lane();
  for (int s = 0; s < a.S; ++s) dma_1k(bs + (size_t)s * a.n_pad + j0 + 4 * lane, sb_lds + s * 1024);
}

template <int S, int NS, int SPB>
__device__ __forceinline__ void screen_block(const MArgs& a, int tb, int split, unsigned char* smem,
                                             float (*sbuf)[kSBRows * kSJ]) {
  static_assert(NS % SPB == 0 && NS / SPB >= 2, "the ring holds at least two groups of stages");
  constexpr int LA = NS / SPB - 1;
  constexpr int L = 2;   // copies per wave per stage
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave / kWJ, wj = wave % kWJ, col = lane & 31, g = lane >> 5;
  const int64_t i0 = (int64_t)tb * kMI;
  const int64_t jb0 = (int64_t)split * a.s_jps;
  const int64_t jb1 = jb0 + a.s_jps < a.n ? jb0 + a.s_jps : a.n;
  const int ntiles = __builtin_amdgcn_readfirstlane(jb1 > jb0 ? (int)((jb1 - jb0 + kSJ - 1) / kSJ) : 0);
  if (ntiles == 0) return;
  const int nchunks = __builtin_amdgcn_readfirstlane(a.rp / kKC);
  const int Q = ntiles * nchunks;
  const unsigned char* gb = reinterpret_cast<const unsigned char*>(a.bf);
  const int64_t n_pad = a.n_pad;
  const uint32_t smem_lds = __builtin_amdgcn_readfirstlane(lds_addr(smem));
  const uint32_t sb_lds = __builtin_amdgcn_readfirstlane(lds_addr(&sbuf[0][0]));
  constexpr uint32_t kSbBytes = kSBRows * kSJ * 4;
  const float* bs = a.bsrc;

  // per target and scale: a_i + hx_i F, the running lower bound of the row
  // maximum (the exact self-pair exponent to start) and the slack of its
  // update (the error of G and twice the bound of the x.f term); per scale the
  // margin (the error of G, the skip depth and 16 bits)
  const double X = a.scal[1], F = a.scal[2];
  const double gam = a.rp * 0x1p-24;
  float at[kIB][S], M[kIB][S], margin[S], slack[kIB][S];
  bool hv[kIB];   // the row counts the pair (i, j*) apart: it is no pair of the verdict
  const int64_t jstar = heavy_source(a);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double XT = X + a.taud[s] * F;
    const double dD = 2.0 * X * (a.eps_g1 + gam) * X + 16.0 * 0x1p-24 * XT * XT;
    margin[s] = (float)(2.0 * a.kapd[s] * dD + (double)kSkip + 16.0);
  }
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
    const bool valid = i < a.n;
    hv[ib] = valid && a.rhv && a.rhv[i] != -INFINITY;
    const double nx = valid ? a.node[i] : 0.0;
    const double nf = valid ? a.node[a.n + i] : 0.0;
    const double nxf = valid ? a.node[2 * a.n + i] : 0.0;
    const float li = valid ? a.lw2[i] : -INFINITY;
    // hx_i F with 2 kap_s tau_s = log2(e) / q for every s, rounded up
    const double hF = 2.0 * a.kapd[0] * a.taud[0] * sqrt(nx) * F * (1.0 + 0x1p-20);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      at[ib][s] = valid ? (float)(-a.kapd[s] * nx + hF) : -INFINITY;
      const float self = (valid && li != -INFINITY) ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf) : -INFINITY;
      M[ib][s] = (valid && a.rref) ? a.rref[(size_t)s * a.n + i] : self;
      slack[ib][s] = (float)((double)margin[s] - kSkip - 15.0 + 2.0 * hF);
    }
  }

  screen_issue_bias(a, bs, sb_lds, jb0, wave);
#pragma unroll
  for (int p = 0; p < LA * SPB; ++p)
    if (p < Q) screen_issue_stage(gb, n_pad, smem_lds + p * kSStage, p % nchunks, i0, jb0 + (int64_t)(p / nchunks) * kSJ,
                                  wave);

  for (int t = 0; t < ntiles; ++t) {
    const int64_t j0 = jb0 + (int64_t)t * kSJ;
    f32x16_t G[kIB][kSJB];
#pragma unroll
    for (int x = 0; x < kIB; ++x)
#pragma unroll
      for (int y = 0; y < kSJB; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) G[x][y][v] = 0.f;
    for (int c = 0; c < nchunks; c += SPB) {
      const int q = t * nchunks + c;
      // this wave's copies of the group have landed (later groups may still fly,
      // unless a tile has so few groups that the copies waited for here were
      // issued before the biases of the tile ending at this group) ...
      if (q + LA * SPB - 1 < Q && 2 * (nchunks / SPB) - 1 >= LA) wait_vmcnt<(LA - 1) * SPB * L>();
      else wait_vmcnt<0>();
      __syncthreads();   // ... for every wave
      if (c == 0 && t + 1 < ntiles) screen_issue_bias(a, bs, sb_lds + ((t + 1) & 1) * kSbBytes, j0 + kSJ, wave);
#pragma unroll
      for (int u = 0; u < SPB; ++u) {
        const int qn = q + LA * SPB + u;
        if (qn < Q) {
          const int tn = qn / nchunks;
          screen_issue_stage(gb, n_pad, smem_lds + (qn % NS) * kSStage, qn - tn * nchunks, i0,
                             jb0 + (int64_t)tn * kSJ, wave);
        }
      }
      SFrag fr[2];
      screen_load_frags(smem + (q % NS) * kSStage, fr[0], wave);
#pragma unroll
      for (int u = 0; u < SPB; ++u) {
        if (u + 1 < SPB) screen_load_frags(smem + ((q + u + 1) % NS) * kSStage, fr[(u + 1) & 1], wave);
        screen_mma(fr[u & 1], G);
      }
    }
    // the verdict on this wave's 64 x 128 sub-tile
    const float* sb = &sbuf[t & 1][0];
    const bool diag = j0 < i0 + kMI && i0 < j0 + kSJ;
    const int jl0 = wj * (32 * kSJB);
    const bool htile = jstar >= j0 + jl0 && jstar < j0 + jl0 + 32 * kSJB;
    bool need = false;
    // slab indices jb * 16 + v in this lane of the self pair and of the pair (i, j*) where the row
    // counts that one apart (-1: none)
    int bself[kIB], bheavy[kIB];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
      bself[ib] = diag ? slab_index<kSJB>(i - j0 - jl0, g) : -1;
      bheavy[ib] = (htile && hv[ib]) ? slab_index<kSJB>(jstar - j0 - jl0, g) : -1;
    }
    // scales outermost: each source bias is read once for both target blocks;
    // the per-target term a_i + hx_i F is added after the maximum, and only a
    // tile that holds self pairs or j* compares slab indices
    auto scan = [&](auto with_self) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float c1 = a.c1[s];
        float m[kIB];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) m[ib] = -INFINITY;
#pragma unroll
        for (int jb = 0; jb < kSJB; ++jb) {
          __builtin_amdgcn_sched_barrier(0);   // one 32-source block's biases in flight at a time
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const float bj = sb[s * kSJ + jl0 + jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3)];
#pragma unroll
            for (int ib = 0; ib < kIB; ++ib) {
              float e = fmaf(c1, G[ib][jb][v], bj);
              if (decltype(with_self)::value && (jb * 16 + v == bself[ib] || jb * 16 + v == bheavy[ib]))
                e = -INFINITY;
              m[ib] = fmaxf(m[ib], e);
            }
          }
        }
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) {
          const float mt = m[ib] + at[ib][s];
          need |= mt > M[ib][s] - margin[s];
          M[ib][s] = fmaxf(M[ib][s], mt - slack[ib][s]);
        }
      }
    };
    // A coarse bound first: max_j (c1 G_ij + b_js) <= c1 max_j G_ij + max_j b_js
    // over the wave's 128 sources; the slab scan runs only if it leaves a doubt
    // in some lane (always on a tile holding self pairs, whose G_ii dominates).
    float gmax[kIB];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      float m = -INFINITY;
#pragma unroll
      for (int jb = 0; jb < kSJB; ++jb)
#pragma unroll
        for (int v = 0; v < 16; ++v) m = fmaxf(m, G[ib][jb][v]);
      gmax[ib] = m;
    }
    // (read through the scalar cache: the address is wave-uniform, and a vector
    // load would make its wait count the stage copies in flight)
    typedef const __attribute__((address_space(4))) float* const_f32_ptr;
    const const_f32_ptr bmax =
        (const_f32_ptr)(bs + (size_t)S * n_pad + (size_t)(j0 / kMJ + wj));   // scale s at s (n_pad / 128)
    bool doubt = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float bm = bmax[(size_t)s * (n_pad / kMJ)];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) doubt |= fmaf(a.c1[s], gmax[ib], bm) + at[ib][s] > M[ib][s] - margin[s];
    }
    if (__any(doubt)) {
      if (diag || htile) scan(std::true_type{});
      else scan(std::false_type{});
    }
    __builtin_amdgcn_sched_barrier(0);
    const bool flag = __any(need);
    const int64_t jt = j0 / kMJ + wj;   // the split pass's 128-source tile of this sub-tile
    if (lane == 0 && jt < a.jtl) {
      a.flags[((size_t)tb * a.jtl + jt) * 8 + wi] = flag ? 1 : 0;
      a.flags[((size_t)tb * a.jtl + jt) * 8 + 4 + wi] = 0;
    }
  }
}

__device__ inline void screen_block_map(const MArgs& a, int& tb, int& split) {
  const int b = blockIdx.x;
  const int per_xcd = a.tb_count / 8;
  if (a.group_t > 0 && per_xcd > 0 && per_xcd * 8 == a.tb_count && per_xcd % a.group_t == 0) {
    const int xcd = b % 8, slot = b / 8;
    const int gsz = a.group_t * a.s_nsplit;
    const int grp = slot / gsz, rem = slot % gsz;
    tb = xcd * per_xcd + grp * a.group_t + rem % a.group_t;
    split = rem / a.group_t;
  } else {
    tb = b / a.s_nsplit;
    split = b % a.s_nsplit;
  }
}

// ---------------------------------------------------------------------------
// The partial-distance screen of BF16X3P as a pipeline of its own.  Its K
// range is PC stages (the first kPreK coordinates), so a wave keeps the hi(x)
// fragments of its 64 targets in registers for the whole block and only the
// sources stream through LDS: one 4 KB stage (128 sources x 16 K values) per
// K chunk, PC stages per tile, a ring of NS stages with LA = NS / PC - 1 tiles
// in flight.  A block is 4 waves (256 targets x 128 sources per tile) and a CU
// runs two, which do not wait for each other at the per-tile barrier.
// The bound: over the first kPreK coordinates (superscript p),
// |x_i - m_j|^2 >= |x_i^p - m_j^p|^2, so the bound of screen_block with G, the
// norms and F taken over those coordinates (a_i^p, b_js^p in a.bpre, F^p)
// bounds the exact exponent from above.  Being no lower bound of the row
// maximum, it leaves M at the row's exact lower bound (the self pair, or the
// pair with the heaviest source where that is larger); boundary targets,
// whose result is -inf whatever the sum, are not flagged.  The source biases
// of a tile are read (through the scalar cache) only when its coarse bound
// leaves a doubt.
constexpr int kPJ = 128;              // sources per tile of the partial-distance screen
constexpr int kPW = kMI / (32 * kIB); // its waves per block (64 targets each)
constexpr int kPStage = kPJ * 32;     // bytes per stage

__device__ inline void prescreen_issue(const unsigned char* gb, int64_t n_pad, uint32_t stage_lds, int c,
                                       int64_t j0, int wave) {
  const int lane = fresh_lane(), rl = lane >> 1, pc = lane & 1;
  const int loff = rl * 32 + swz<2>(rl, pc) * 16;
  dma_1k(gb + ((uint64_t)c * (uint64_t)n_pad + (uint64_t)(j0 + wave * 32)) * 32 + loff, stage_lds + wave * 1024);
}

template <int S, int PC, int NS>
__device__ __forceinline__ void prescreen_block(const MArgs& a, int tb, int split, unsigned char* smem) {
  static_assert(NS % PC == 0 && NS / PC >= 2, "the ring holds at least two tiles");
  static_assert(PC * kKC <= kPreK, "the screen covers the first kPreK coordinates");
  static_assert(kPW * 32 == kPJ && kSJB * 32 == kPJ, "one 1 KB copy per wave per stage; a wave spans the tile");
  constexpr int LA = NS / PC - 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave, col = lane & 31, g = lane >> 5;
  const int64_t i0 = (int64_t)tb * kMI;
  const int64_t jb0 = (int64_t)split * a.s_jps;
  const int64_t jb1 = jb0 + a.s_jps < a.n ? jb0 + a.s_jps : a.n;
  const int ntiles = __builtin_amdgcn_readfirstlane(jb1 > jb0 ? (int)((jb1 - jb0 + kPJ - 1) / kPJ) : 0);
  if (ntiles == 0) return;
  const unsigned char* gb = reinterpret_cast<const unsigned char*>(a.bf);
  const int64_t n_pad = a.n_pad;
  const uint32_t smem_lds = __builtin_amdgcn_readfirstlane(lds_addr(smem));

  // per target and scale: a_i^p + hx_i^p F^p and the exact self-pair exponent;
  // per scale the margin (as in screen_block, over the first PC stages)
  const double X = a.scal[4], F = a.scal[5];
  const double gam = PC * kKC * 0x1p-24;
  float at[kIB][S], M[kIB][S], margin[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double XT = X + a.taud[s] * F;
    const double dD = 2.0 * X * (a.eps_g1 + gam) * X + 16.0 * 0x1p-24 * XT * XT;
    margin[s] = (float)(2.0 * a.kapd[s] * dD + (double)kSkip + 16.0);
  }
  // the targets' fragments, all PC stages (rows i0 .. i0 + 255 < n_pad)
  bf16x8_t bt[PC][kIB];
  bool hv[kIB];   // the row counts the pair (i, j*) apart: it is no pair of the verdict
  const int64_t jstar = heavy_source(a);
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
    const bool valid = i < a.n && !a.bnd[i];
    hv[ib] = valid && a.rhv && a.rhv[i] != -INFINITY;
    const double nx = valid ? a.node[3 * a.n + i] : 0.0;
    const double nf = valid ? a.node[a.n + i] : 0.0;
    const float li = valid ? a.lw2[i] : -INFINITY;
    const double hF = 2.0 * a.kapd[0] * a.taud[0] * sqrt(nx) * F * (1.0 + 0x1p-20);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      at[ib][s] = valid ? (float)(-a.kapd[s] * nx + hF) : -INFINITY;
      const float self = (valid && li != -INFINITY) ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf) : -INFINITY;
      M[ib][s] = (valid && a.rref) ? a.rref[(size_t)s * a.n + i] : self;
    }
#pragma unroll
    for (int c = 0; c < PC; ++c)
      bt[c][ib] = *reinterpret_cast<const bf16x8_t*>(gb + ((size_t)c * n_pad + i) * 32 + g * 16);
  }
  // per scale the largest prefix bias over the block's source range (the tiles' maxima, lane-parallel):
  // a coarse bound that needs no load inside the tile loop
  typedef const __attribute__((address_space(4))) float* const_f32_ptr;
  const float* tmax = a.bpre + (size_t)S * n_pad;   // [S][n_pad / 128] the tiles' maxima
  float bblk[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float m = -INFINITY;
    for (int t = lane; t < ntiles; t += 64) m = fmaxf(m, tmax[(size_t)s * (n_pad / kMJ) + (size_t)(jb0 / kMJ) + t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    bblk[s] = m;
  }
  wait_vmcnt<0>();   // before the first copy: the waits below count copies only

#pragma unroll
  for (int p = 0; p < LA; ++p)
    if (p < ntiles)
#pragma unroll
      for (int u = 0; u < PC; ++u)
        prescreen_issue(gb, n_pad, smem_lds + ((p * PC + u) % NS) * kPStage, u, jb0 + (int64_t)p * kPJ, wave);

  for (int t = 0; t < ntiles; ++t) {
    const int64_t j0 = jb0 + (int64_t)t * kPJ;
    // this wave's copies of tile t have landed (those of the next LA - 1 tiles may still fly) ...
    if (t + LA - 1 < ntiles) wait_vmcnt<(LA - 1) * PC>();
    else wait_vmcnt<0>();
    __syncthreads();   // ... for every wave; the slots of tile t - 1 are free again
    if (t + LA < ntiles)
#pragma unroll
      for (int u = 0; u < PC; ++u)
        prescreen_issue(gb, n_pad, smem_lds + (((t + LA) * PC + u) % NS) * kPStage, u, j0 + (int64_t)LA * kPJ,
                        wave);
    f32x16_t G[kIB][kSJB];
#pragma unroll
    for (int x = 0; x < kIB; ++x)
#pragma unroll
      for (int y = 0; y < kSJB; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) G[x][y][v] = 0.f;
#pragma unroll
    for (int u = 0; u < PC; ++u) {
      const unsigned char* base = smem + ((t * PC + u) % NS) * kPStage;
      const int ln = fresh_lane(), cl = ln & 31, gl = ln >> 5;
      bf16x8_t xh[kSJB];
#pragma unroll
      for (int jb = 0; jb < kSJB; ++jb) {
        const int row = jb * 32 + cl;
        xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + row * 32 + swz<2>(row, gl) * 16);
      }
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < kSJB; ++jb)
          G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bt[u][ib], G[ib][jb], 0, 0, 0);
    }
    // the verdict on this wave's 64 x 128 sub-tile: the coarse bound, then the
    // per-pair bound where it leaves a doubt
    const bool diag = j0 < i0 + kMI && i0 < j0 + kPJ;
    float gmax[kIB];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      float m = -INFINITY;
#pragma unroll
      for (int jb = 0; jb < kSJB; ++jb)
#pragma unroll
        for (int v = 0; v < 16; ++v) m = fmaxf(m, G[ib][jb][v]);
      gmax[ib] = m;
    }
    // the coarse bound with the block's largest bias first, then with the tile's
    bool doubt = false;
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) doubt |= fmaf(a.c1[s], gmax[ib], bblk[s]) + at[ib][s] > M[ib][s] - margin[s];
    if (__any(doubt)) {
      const const_f32_ptr bmax = (const_f32_ptr)(tmax + (size_t)(j0 / kMJ));
      doubt = false;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float bm = bmax[(size_t)s * (n_pad / kMJ)];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) doubt |= fmaf(a.c1[s], gmax[ib], bm) + at[ib][s] > M[ib][s] - margin[s];
      }
    }
    bool need = false;
    if (__any(doubt)) {
      // slab indices jb * 16 + v in this lane of the self pair and of the pair (i, j*) where the row
      // counts that one apart (-1: none)
      const bool htile = jstar >= j0 && jstar < j0 + kPJ;
      int bself[kIB], bheavy[kIB];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) {
        const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
        bself[ib] = diag ? slab_index<kSJB>(i - j0, g) : -1;
        bheavy[ib] = (htile && hv[ib]) ? slab_index<kSJB>(jstar - j0, g) : -1;
      }
      // (the biases through the scalar cache: the addresses are wave-uniform
      // up to the lane half g, and a vector load would wait for the copies)
      typedef float f32x8_t __attribute__((ext_vector_type(8)));
      typedef const __attribute__((address_space(4))) f32x8_t* const_f32x8_ptr;
      const const_f32x8_ptr bs = (const_f32x8_ptr)(a.bpre + j0);   // 8 sources per element
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float c1 = a.c1[s];
        float m[kIB];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) m[ib] = -INFINITY;
#pragma unroll
        for (int jb = 0; jb < kSJB; ++jb) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            // sources 8 (v >> 2) + 4 g + (v & 3) of the 32-source block jb
            const f32x8_t q = bs[((size_t)s * n_pad) / 8 + jb * 4 + (v >> 2)];
            const float bj = g ? q[4 + (v & 3)] : q[v & 3];
#pragma unroll
            for (int ib = 0; ib < kIB; ++ib) {
              float e = fmaf(c1, G[ib][jb][v], bj);
              if (jb * 16 + v == bself[ib] || jb * 16 + v == bheavy[ib]) e = -INFINITY;
              m[ib] = fmaxf(m[ib], e);
            }
          }
        }
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) need |= m[ib] + at[ib][s] > M[ib][s] - margin[s];
      }
    }
    const bool flag = __any(need);
    const int64_t jt = j0 / kMJ;   // the split pass's 128-source tile
    if (lane == 0 && jt < a.jtl) {
      a.flags[((size_t)tb * a.jtl + jt) * 8 + wi] = flag ? 1 : 0;
      a.flags[((size_t)tb * a.jtl + jt) * 8 + 4 + wi] = 0;
      if (flag && a.any_flag) *a.any_flag = 1;
    }
  }
}

// The symmetric partial-distance screen.  G^p = X^p X^p^T is symmetric, so one
// block of products between target blocks A and B (A < B) serves both
// orientations: A's rows against B's sources, with the per-row verdict of
// prescreen_block, and B's rows against A's sources, with a coarse bound per
// (wave, 64 rows of B): for row j of B and source i of the wave's 64 nodes of A,
//   e_ji <= a_j + c1 G_ij + b_i <= c1 max_(wave x group) G + max_i b_i + max_j (a_j - M_j) + M_j,
// so no row j of the group is within the margin of its lower bound M_j unless
// c1 max G + max b + max (a - M) > -margin.  The rows that count the pair with
// the heaviest source j* apart take max b over the wave's sources without j*.
// Work items (A, B0, B1) cover every unordered pair of target blocks once (the
// diagonal A = B with the per-row verdict only), and each flag byte is written
// by exactly one wave per call: (A, tiles of B >= A) in the normal orientation,
// (B, tiles of A < B) in the transposed one.
//
// Where that coarse bound leaves a doubt, the unit (B, group, A, wave) goes to a
// list, and k_sym_recheck takes the group's rows against the wave's sources one
// by one with the per-row verdict, after the screen.
//
// k_tgt_bound: per 64-row group and scale the largest a_j^p + hx_j^p F^p - M_j over
// the group's rows, split by whether the row counts the heavy pair apart (a_j is
// the screen's target term, M_j the row's lower bound as the screens take it);
// and it clears the list's counter.
__device__ __forceinline__ void tgt_bound_body(const MArgs& a, int bx) {
  const int lane = threadIdx.x & 63;
  const int g = (int)(((int64_t)bx * kBlock + threadIdx.x) >> 6);
  if (bx == 0 && threadIdx.x == 0) *a.sym_n = 0;
  if (g >= a.ngroups) return;   // whole waves: ngroups groups of 64 rows
  const int64_t j = (int64_t)g * 64 + lane;
  const double F = a.scal[5];
  const bool valid = j < a.n && !a.bnd[j];
  const double nx = valid ? a.node[3 * a.n + j] : 0.0;
  const double nf = valid ? a.node[a.n + j] : 0.0;
  const float li = valid ? a.lw2[j] : -INFINITY;
  const bool hv = valid && a.rhv && a.rhv[j] != -INFINITY;
  const double hF = 2.0 * a.kapd[0] * a.taud[0] * sqrt(nx) * F * (1.0 + 0x1p-20);
  float* out = const_cast<float*>(a.tT);
  for (int s = 0; s < a.S; ++s) {
    float v = -INFINITY;
    if (valid) {
      const float at = (float)(-a.kapd[s] * nx + hF);
      const float self = li != -INFINITY ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf) : -INFINITY;
      const float M = a.rref ? a.rref[(size_t)s * a.n + j] : self;
      v = at - M;   // +inf where M = -inf: any pair may then be near
    }
    float vh = hv ? v : -INFINITY, vn = hv ? -INFINITY : v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      vh = fmaxf(vh, __shfl_xor(vh, off, 64));
      vn = fmaxf(vn, __shfl_xor(vn, off, 64));
    }
    if (lane == 0) {
      out[(size_t)s * a.ngroups + g] = vh;
      out[(size_t)(a.S + s) * a.ngroups + g] = vn;
    }
  }
}
__global__ void __launch_bounds__(kBlock) k_tgt_bound(MArgs a) { tgt_bound_body(a, blockIdx.x); }
// batched: items (run, block of the run's launch)
__global__ void __launch_bounds__(kBlock) k_tgt_bound_batch(const MArgs* __restrict__ sets,
                                                            const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  tgt_bound_body(sets[__builtin_amdgcn_readfirstlane(it.x)], __builtin_amdgcn_readfirstlane(it.y));
}

// DPP moves within rows of 16 lanes (quad_perm and row_ror controls): every lane gets the largest value of
// its row; with the four rows' lanes 0 read as scalars a wave is reduced without the LDS permute path.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp_mov<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  v = fmaxf(v, dpp_mov<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  v = fmaxf(v, dpp_mov<0x124>(v));   // row_ror 4
  return fmaxf(v, dpp_mov<0x128>(v));   // row_ror 8
}
__device__ __forceinline__ float lane_of(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// The partial-distance screen's per-scale margin over its first PC stages, and per target row i its term
// a_i^p + hx_i^p F^p, the lower bound M_i of its maximum (the row floor, else the self-pair exponent)
// and whether it counts the pair with the heaviest source apart.
template <int S, int PC>
__device__ __forceinline__ void screen_margins(const MArgs& a, float (&margin)[S]) {
  const double X = a.scal[4], F = a.scal[5];
  const double gam = PC * kKC * 0x1p-24;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double XT = X + a.taud[s] * F;
    const double dD = 2.0 * X * (a.eps_g1 + gam) * X + 16.0 * 0x1p-24 * XT * XT;
    margin[s] = (float)(2.0 * a.kapd[s] * dD + (double)kSkip + 16.0);
  }
}
template <int S>
__device__ __forceinline__ bool screen_target(const MArgs& a, int64_t i, float (&at)[S], float (&M)[S]) {
  const double F = a.scal[5];
  const bool valid = i < a.n && !a.bnd[i];
  const double nx = valid ? a.node[3 * a.n + i] : 0.0;
  const double nf = valid ? a.node[a.n + i] : 0.0;
  const float li = valid ? a.lw2[i] : -INFINITY;
  const double hF = 2.0 * a.kapd[0] * a.taud[0] * sqrt(nx) * F * (1.0 + 0x1p-20);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    at[s] = valid ? (float)(-a.kapd[s] * nx + hF) : -INFINITY;
    const float self = (valid && li != -INFINITY) ? li - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * nf) : -INFINITY;
    M[s] = (valid && a.rref) ? a.rref[(size_t)s * a.n + i] : self;
  }
  return valid && a.rhv && a.rhv[i] != -INFINITY;
}

template <int S, int PC, int NS>
__device__ __forceinline__ void prescreen_sym_block(const MArgs& a, int A, int B0, int B1, unsigned char* smem,
                                                    uint8_t (*sbits)[4][4], float* stT,
                                                    double (*slim)[2][S]) {
  static_assert(NS % PC == 0 && NS / PC >= 2, "the ring holds at least two tiles");
  static_assert(PC * kKC <= kPreK, "the screen covers the first kPreK coordinates");
  static_assert(kPW == 4 && kPW * 32 == kPJ && kSJB * 32 == kPJ, "4 waves of 64 targets; a wave spans the tile");
  constexpr int LA = NS / PC - 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave, col = lane & 31, g = lane >> 5;
  const int64_t i0 = (int64_t)A * kMI;
  const int jt0 = 2 * B0;
  const int jt1 = (int)(2 * (int64_t)B1 < a.jtl ? 2 * (int64_t)B1 : a.jtl);
  const int ntiles = __builtin_amdgcn_readfirstlane(jt1 - jt0);
  if (ntiles <= 0) return;
  const unsigned char* gb = reinterpret_cast<const unsigned char*>(a.bf);
  const int64_t n_pad = a.n_pad;
  const uint32_t smem_lds = __builtin_amdgcn_readfirstlane(lds_addr(smem));

  float at[kIB][S], M[kIB][S], margin[S];
  screen_margins<S, PC>(a, margin);
  bf16x8_t bt[PC][kIB];
  bool hv[kIB];
  const int64_t jstar = heavy_source(a);
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
    hv[ib] = screen_target<S>(a, i, at[ib], M[ib]);
#pragma unroll
    for (int c = 0; c < PC; ++c)
      bt[c][ib] = *reinterpret_cast<const bf16x8_t*>(gb + ((size_t)c * n_pad + i) * 32 + g * 16);
  }
  // the transposed orientation: the wave's 64 nodes of A as sources, their largest prefix bias with
  // and without j*
  float bA[S], bAx[S];
  {
    const int64_t i = i0 + wi * 64 + lane;   // < n_pad
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float v = a.bpre[(size_t)s * n_pad + i], vx = i == jstar ? -INFINITY : v;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        v = fmaxf(v, __shfl_xor(v, off, 64));
        vx = fmaxf(vx, __shfl_xor(vx, off, 64));
      }
      bA[s] = v;
      bAx[s] = vx;
    }
  }
  // the transposed check's limits per wave in LDS, read after each tile's barrier (kept in registers they
  // would be spilled, and the reload would wait for every copy in flight): -(margin + 1) less the
  // wave's largest source bias, with j* left out and with it
  if (lane == 0)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double lim = -((double)margin[s] + 1.0);
      slim[wi][0][s] = lim - (double)bAx[s];
      slim[wi][1][s] = lim - (double)bA[s];
    }
  typedef const __attribute__((address_space(4))) float* const_f32_ptr;
  const float* tmax = a.bpre + (size_t)S * n_pad;   // [S][n_pad / 128] the tiles' maxima
  float bblk[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float m = -INFINITY;
    for (int t = lane; t < ntiles; t += 64) m = fmaxf(m, tmax[(size_t)s * (n_pad / kMJ) + (size_t)jt0 + t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    bblk[s] = m;
  }
  // the group bounds of the block's sources (B0 .. B1, 4 groups each) into LDS: stT[(c S + s) 4 kSymChunk + k]
  {
    const int ng = 4 * (B1 - B0);   // <= 4 kSymChunk
    for (int e = threadIdx.x; e < 2 * S * ng; e += kPW * 64) {
      const int cs = e / ng, k = e % ng;
      stT[cs * 4 * kSymChunk + k] = a.tT[(size_t)cs * a.ngroups + 4 * B0 + k];
    }
  }
  wait_vmcnt<0>();   // before the first copy: the waits below count copies only (the first tile's barrier
                     // publishes stT)

#pragma unroll
  for (int p = 0; p < LA; ++p)
    if (p < ntiles)
#pragma unroll
      for (int u = 0; u < PC; ++u)
        prescreen_issue(gb, n_pad, smem_lds + ((p * PC + u) % NS) * kPStage, u, (int64_t)(jt0 + p) * kPJ, wave);

  bool anyT = false;
  // writes the flag entries (B, 2A) and (B, 2A + 1) from the waves' bits of B (wave 0, after a barrier)
  // (the lane index is formed afresh here: a value kept from the kernel's start would be spilled, and
  // its reload would wait for every copy in flight)
  auto store_transposed = [&](int B) {
    if (wave == 0) {
      const int h = fresh_lane();   // A's source tile 2A + h: waves 2h and 2h + 1
      if (h < 2) {
        const uint8_t(*sb)[4] = sbits[B & 1];
        uint64_t v = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) v |= (uint64_t)(sb[2 * h][w] | sb[2 * h + 1][w]) << (8 * w);
        *reinterpret_cast<uint64_t*>(a.flags + ((size_t)B * a.jtl + 2 * A + h) * 8) = v;
      }
    }
  };
  for (int t = 0; t < ntiles; ++t) {
    const int jt = jt0 + t;
    const int64_t j0 = (int64_t)jt * kPJ;
    const int B = jt >> 1, hB = jt & 1;
    if (t + LA - 1 < ntiles) wait_vmcnt<(LA - 1) * PC>();
    else wait_vmcnt<0>();
    __syncthreads();   // the copies of tile t have landed for every wave; the bits of the B before last are read
    if (hB == 0 && B - 1 > A && B - 1 >= B0) store_transposed(B - 1);
    if (t + LA < ntiles)
#pragma unroll
      for (int u = 0; u < PC; ++u)
        prescreen_issue(gb, n_pad, smem_lds + (((t + LA) * PC + u) % NS) * kPStage, u, j0 + (int64_t)LA * kPJ, wave);
    f32x16_t G[kIB][kSJB];
#pragma unroll
    for (int x = 0; x < kIB; ++x)
#pragma unroll
      for (int y = 0; y < kSJB; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) G[x][y][v] = 0.f;
#pragma unroll
    for (int u = 0; u < PC; ++u) {
      const unsigned char* base = smem + ((t * PC + u) % NS) * kPStage;
      const int ln = fresh_lane(), cl = ln & 31, gl = ln >> 5;
      bf16x8_t xh[kSJB];
#pragma unroll
      for (int jb = 0; jb < kSJB; ++jb) {
        const int row = jb * 32 + cl;
        xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + row * 32 + swz<2>(row, gl) * 16);
      }
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < kSJB; ++jb)
          G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bt[u][ib], G[ib][jb], 0, 0, 0);
    }
    // the lane's maxima of G per (node block ib, source half q): both orientations' coarse bounds
    // take them, so that the tile's values are scanned once
    float pm[kIB][2];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float m = -INFINITY;
#pragma unroll
        for (int jb = 2 * q; jb < 2 * q + 2; ++jb)
#pragma unroll
          for (int v = 0; v < 16; ++v) m = fmaxf(m, G[ib][jb][v]);
        pm[ib][q] = m;
      }
    // (1) A's rows against this tile's sources: as prescreen_block
    const bool diag = j0 < i0 + kMI && i0 < j0 + kPJ;
    float gmax[kIB];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) gmax[ib] = fmaxf(pm[ib][0], pm[ib][1]);
    bool doubt = false;
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) doubt |= fmaf(a.c1[s], gmax[ib], bblk[s]) + at[ib][s] > M[ib][s] - margin[s];
    if (__any(doubt)) {
      const const_f32_ptr bmax = (const_f32_ptr)(tmax + (size_t)jt);
      doubt = false;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float bm = bmax[(size_t)s * (n_pad / kMJ)];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) doubt |= fmaf(a.c1[s], gmax[ib], bm) + at[ib][s] > M[ib][s] - margin[s];
      }
    }
    bool need = false;
    if (__any(doubt)) {
      const bool htile = jstar >= j0 && jstar < j0 + kPJ;
      int bself[kIB], bheavy[kIB];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) {
        const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
        bself[ib] = diag ? slab_index<kSJB>(i - j0, g) : -1;
        bheavy[ib] = (htile && hv[ib]) ? slab_index<kSJB>(jstar - j0, g) : -1;
      }
      typedef float f32x8_t __attribute__((ext_vector_type(8)));
      typedef const __attribute__((address_space(4))) f32x8_t* const_f32x8_ptr;
      const const_f32x8_ptr bs = (const_f32x8_ptr)(a.bpre + j0);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float c1 = a.c1[s];
        float m[kIB];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) m[ib] = -INFINITY;
#pragma unroll
        for (int jb = 0; jb < kSJB; ++jb) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const f32x8_t q = bs[((size_t)s * n_pad) / 8 + jb * 4 + (v >> 2)];
            const float bj = g ? q[4 + (v & 3)] : q[v & 3];
#pragma unroll
            for (int ib = 0; ib < kIB; ++ib) {
              float e = fmaf(c1, G[ib][jb][v], bj);
              if (jb * 16 + v == bself[ib] || jb * 16 + v == bheavy[ib]) e = -INFINITY;
              m[ib] = fmaxf(m[ib], e);
            }
          }
        }
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) need |= m[ib] + at[ib][s] > M[ib][s] - margin[s];
      }
    }
    const bool flag = __any(need);
    if (lane == 0 && jt < a.jtl) {
      a.flags[((size_t)A * a.jtl + jt) * 8 + wi] = flag ? 1 : 0;
      a.flags[((size_t)A * a.jtl + jt) * 8 + 4 + wi] = 0;
      if (flag && a.any_flag) *a.any_flag = 1;
    }
    // (2) B's rows (sub-blocks 2 hB and 2 hB + 1) against the wave's 64 sources of A: the coarse bound
    if (B != A) {
      float gm[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float m = -INFINITY;
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) m = fmaxf(m, pm[ib][q]);
        m = row16_max(m);
        gm[q] = fmaxf(fmaxf(lane_of(m, 0), lane_of(m, 16)), fmaxf(lane_of(m, 32), lane_of(m, 48)));
      }
      // (the groups' bounds from LDS: a load from memory here would wait for the copies in flight)
      bool fq[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = (B - B0) * 4 + 2 * hB + q;   // B's 64-row group, within the block's sources
        bool f = false;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          // in FP64, with one bit of slack for the terms' own FP32 rounding
          const double th = stT[s * 4 * kSymChunk + k], tn = stT[(S + s) * 4 * kSymChunk + k];
          const double cg = (double)a.c1[s] * (double)gm[q];
          f |= cg + th > slim[wi][0][s];
          f |= cg + tn > slim[wi][1][s];
        }
        fq[q] = f;
      }

      // where the bound doubts, the group's rows go to k_sym_recheck (its flag byte stays 0 here; with
      // the list full, the group is flagged)
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          bool bit = false;
          if (fq[q]) {
            const int u = atomicAdd(a.sym_n, 1);
            if (u < a.sym_cap) a.sym_list[u] = make_int4(B, 2 * hB + q, A, wi);
            else bit = true;
          }
          sbits[B & 1][wi][2 * hB + q] = bit ? 1 : 0;
          anyT |= bit;
        }
        if (hB == 0 && jt + 1 >= a.jtl) {   // B's second tile lies past the last node: its rows are empty
          sbits[B & 1][wi][2] = 0;
          sbits[B & 1][wi][3] = 0;
        }
      }
    }
  }
  __syncthreads();
  {
    const int Bl = (jt1 - 1) >> 1;
    if (Bl > A) store_transposed(Bl);
  }
  if (anyT && a.any_flag) *a.any_flag = 1;
}

template <int S, int PC, int NS>
__global__ void __launch_bounds__(kPW * 64, 2) k_pair_prescreen_sym(MArgs a) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * kPStage];
  __shared__ uint8_t sbits[2][4][4];
  __shared__ float stT[2 * S * 4 * kSymChunk];
  __shared__ double slim[kPW][2][S];
  const int4 it = a.sym_items[blockIdx.x];
  prescreen_sym_block<S, PC, NS>(a, __builtin_amdgcn_readfirstlane(it.x), __builtin_amdgcn_readfirstlane(it.y),
                                 __builtin_amdgcn_readfirstlane(it.z), smem, sbits, stT, slim);
}

// The units where the symmetric screen's coarse bound doubted, row by row in the normal orientation: the 64
// rows of group grp of target block B against the 64 sources that wave wi of target block A holds, from
// the same BF16 products over the first PC stages of coordinates (recomputed here), with
// prescreen_block's per-row verdict (B > A, so no self pair; a row that counts j* apart leaves it out).
// A flagged unit sets its byte of the flag entry (B, source tile 2A + wi / 2).  A wave per unit, the grid
// striding over the list.
template <int S, int PC>
__device__ __forceinline__ void sym_recheck_body(const MArgs& a, int bx, int nblocks) {
  const int nu = __builtin_amdgcn_readfirstlane(min(*a.sym_n, a.sym_cap));
  const int lane = threadIdx.x & 63, col = lane & 31, g = lane >> 5;
  const int nw = nblocks * kPW;
  int u = __builtin_amdgcn_readfirstlane(bx * kPW + (int)(threadIdx.x >> 6));
  if (u >= nu) return;
  const unsigned char* gb = reinterpret_cast<const unsigned char*>(a.bf);
  const int64_t n_pad = a.n_pad;
  float margin[S];
  screen_margins<S, PC>(a, margin);
  const int64_t jstar = heavy_source(a);
  for (; u < nu; u += nw) {
    const int4 e = a.sym_list[u];
    const int B = __builtin_amdgcn_readfirstlane(e.x), grp = __builtin_amdgcn_readfirstlane(e.y);
    const int A = __builtin_amdgcn_readfirstlane(e.z), wi = __builtin_amdgcn_readfirstlane(e.w);
    const int64_t t0 = (int64_t)B * kMI + grp * 64, s0 = (int64_t)A * kMI + wi * 64;
    float at[kIB][S], M[kIB][S];
    bool hv[kIB];
    bf16x8_t bt[PC][kIB], xs[PC][2];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = t0 + ib * 32 + col;
      hv[ib] = screen_target<S>(a, i, at[ib], M[ib]);
#pragma unroll
      for (int c = 0; c < PC; ++c)
        bt[c][ib] = *reinterpret_cast<const bf16x8_t*>(gb + ((size_t)c * n_pad + i) * 32 + g * 16);
    }
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int c = 0; c < PC; ++c)
        xs[c][jb] = *reinterpret_cast<const bf16x8_t*>(gb + ((size_t)c * n_pad + s0 + jb * 32 + col) * 32 + g * 16);
    f32x16_t G[kIB][2];
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
#pragma unroll
        for (int v = 0; v < 16; ++v) G[ib][jb][v] = 0.f;
#pragma unroll
        for (int c = 0; c < PC; ++c) G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xs[c][jb], bt[c][ib], G[ib][jb], 0, 0, 0);
      }
    bool need = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float c1 = a.c1[s];
#pragma unroll
      for (int ib = 0; ib < kIB; ++ib) {
        float m = -INFINITY;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t j = s0 + jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
            float ev = fmaf(c1, G[ib][jb][v], a.bpre[(size_t)s * n_pad + j]);
            if (hv[ib] && j == jstar) ev = -INFINITY;
            m = fmaxf(m, ev);
          }
        need |= m + at[ib][s] > M[ib][s] - margin[s];
      }
    }
    if (__any(need) && lane == 0) {
      a.flags[((size_t)B * a.jtl + 2 * A + (wi >> 1)) * 8 + grp] = 1;
      if (a.any_flag) *a.any_flag = 1;
    }
  }
}
template <int S, int PC>
__global__ void __launch_bounds__(kPW * 64) k_sym_recheck(MArgs a) {
  sym_recheck_body<S, PC>(a, blockIdx.x, gridDim.x);
}
// batched: items (run, block b of the run's nb blocks, nb)
template <int S>
__global__ void __launch_bounds__(kPW * 64) k_sym_recheck_batch(const MArgs* __restrict__ sets,
                                                                const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const MArgs& a = sets[__builtin_amdgcn_readfirstlane(it.x)];
  const int b = __builtin_amdgcn_readfirstlane(it.y), nb = __builtin_amdgcn_readfirstlane(it.z);
  sym_recheck_body<S, 4>(a, b, nb);   // four K stages (host rule)
}

template <int S, int PC, int NS>
__global__ void __launch_bounds__(kPW * 64, 2) k_pair_prescreen(MArgs a) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * kPStage];
  int tb, split;
  screen_block_map(a, tb, split);
  prescreen_block<S, PC, NS>(a, tb, split, smem);
}

// Many node sets: block b takes work item items[b] = (set, target block,
// source split) of the split pass; 4 or 2 K stages as the set's K padding
// allows, 3 tiles in flight either way.
// Items of two kinds: (run, A, B0, B1) with B1 > 0, a symmetric-screen item of a run with more than
// kSymMinBlocks target blocks and r_p > 32; (run, target block, source split, -1), a one-sided one.
template <int S>
__global__ void __launch_bounds__(kPW * 64, 2) k_pair_prescreen_batch(const MArgs* __restrict__ sets,
                                                                      const int4* __restrict__ items) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[16 * kPStage];
  __shared__ uint8_t sbits[2][4][4];
  __shared__ float stT[2 * S * 4 * kSymChunk];
  __shared__ double slim[kPW][2][S];
  const int4 it = items[blockIdx.x];
  const MArgs& a = sets[__builtin_amdgcn_readfirstlane(it.x)];
  const int y = __builtin_amdgcn_readfirstlane(it.y), z = __builtin_amdgcn_readfirstlane(it.z);
  const int w = __builtin_amdgcn_readfirstlane(it.w);
  const bool k4 = __builtin_amdgcn_readfirstlane(a.pre_chunks) == 4;
  if (w > 0) {
    prescreen_sym_block<S, 4, 16>(a, y, z, w, smem, sbits, stT, slim);   // four K stages (host rule)
  } else {
    if (k4) prescreen_block<S, 4, 16>(a, y, z, smem);
    else prescreen_block<S, 2, 8>(a, y, z, smem);
  }
}


template <int S, int NS, int SPB>
__global__ void __launch_bounds__(kNT, 1) k_pair_screen(MArgs a) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * kSStage];
  __shared__ __attribute__((aligned(1024))) float sbuf[2][kSBRows * kSJ];
  int tb, split;
  screen_block_map(a, tb, split);
  screen_block<S, NS, SPB>(a, tb, split, smem, sbuf);
}

template <int S, int NS, int SPB>
__global__ void __launch_bounds__(kNT, 1) k_pair_screen_batch(const MArgs* __restrict__ sets,
                                                              const int4* __restrict__ items) {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[NS * kSStage];
  __shared__ __attribute__((aligned(1024))) float sbuf[2][kSBRows * kSJ];
  const int4 it = items[blockIdx.x];
  screen_block<S, NS, SPB>(sets[__builtin_amdgcn_readfirstlane(it.x)], __builtin_amdgcn_readfirstlane(it.y),
                           __builtin_amdgcn_readfirstlane(it.z), smem, sbuf);
}

// ---------------------------------------------------------------------------
// Source biases b_js = lw2_j - kap_s |m_j^s|^2 (push form; pull form lw2_j -
// kap_s |x_j|^2) (FP64 -> FP32), -inf for invalid
// sources: out[s][n_pad]; then the maximum over each 128 consecutive sources,
// out[S n_pad + s (n_pad / 128) + block] (the screen's coarse bound).  With
// a.bpre the same over the first kPreK coordinates, to a.bpre in the same
// layout.  n_pad is a multiple of the 256 threads of a block.
// (the argument set by reference: in the batched kernel it lives in global memory, and a copy would be
// private memory on every lane)
__device__ __forceinline__ void k_src_bias_body(int64_t n, int64_t n_pad, int32_t S,
                                                     const MArgs& a, float* __restrict__ out, int bx_, int gx_) {
  __shared__ double sh[kBlock / 64];
  const int64_t j = (int64_t)bx_ * kBlock + threadIdx.x;
  if (a.any_flag && bx_ == 0 && threadIdx.x == 0) *a.any_flag = 0;
  for (int part = 0; part < (a.bpre ? 2 : 1); ++part) {
    float* o = part == 0 ? out : const_cast<float*>(a.bpre);
    const double* nd = a.node + (part == 0 ? 0 : 3 * n);
    for (int s = 0; s < S; ++s) {
      float v = -INFINITY;
      if (j < n) {
        const float l = a.lw2[j];
        if (l != -INFINITY) {
          const double t = a.taud[s];
          const double nm = a.pull ? nd[j] : nd[j] + 2.0 * t * nd[2 * n + j] + t * t * nd[n + j];
          v = (float)((double)l - a.kapd[s] * nm);
        }
      }
      if (j < n_pad) o[(size_t)s * n_pad + j] = v;
      const double wm = wave_max((double)v);
      if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = wm;
      __syncthreads();
      if (threadIdx.x < 2 && (int64_t)bx_ * kBlock + 128 * threadIdx.x < n_pad)
        o[(size_t)S * n_pad + (size_t)s * (n_pad / 128) + (size_t)bx_ * 2 + threadIdx.x] =
            (float)fmax(sh[2 * threadIdx.x], sh[2 * threadIdx.x + 1]);
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_src_bias(int64_t n, int64_t n_pad, int32_t S,
                                                     MArgs a, float* __restrict__ out) {
  k_src_bias_body(n, n_pad, S, a, out, blockIdx.x, gridDim.x);
}

// Blocks [0, nbias): the source biases; block nbias: j* and f(x_j*).
__global__ void __launch_bounds__(kBlock) k_src_bias_heavy(int64_t n, int64_t n_pad, int32_t S, MArgs a,
                                                           float* __restrict__ out, RowRefArgs ra, int nbias) {
  if ((int)blockIdx.x < nbias) k_src_bias_body(n, n_pad, S, a, out, blockIdx.x, nbias);
  else k_heavy_body(ra);
}

__global__ void __launch_bounds__(kBlock) k_src_bias_batch(const MArgs* __restrict__ sets, const int* __restrict__ pre,
                                                           int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const MArgs& a = sets[q];
  k_src_bias_body(a.n, a.n_pad, a.S, a, const_cast<float*>(a.bsrc), blockIdx.x - pre[q], pre[q + 1] - pre[q]);
}


int64_t pair_mfma_npad(int64_t n) { return ((n + kMI - 1) / kMI) * kMI; }

static MArgs make_args(const PairArgs& pa, int prec, const MfmaExtra& ex) {
  MArgs m{};
  m.pull = pa.pull;
  m.n = pa.n;
  m.n_pad = ex.n_pad;
  m.r = pa.r;
  m.rp = pa.rp;
  m.S = pa.S;
  // hi/lo split product: 2^-16 per operand split plus cross terms; hi only:
  // 2^-8 per operand; FP32 operands: 2^-24 per operand (rounded up).
  // The screened split form: the BF16X3G bounds, and the one-product bound of G for its screen.
  const bool screened = prec == YY_PREC_BF16X3S || prec == YY_PREC_BF16X3P;
  const bool split_g = prec == YY_PREC_BF16X3 || prec == YY_PREC_BF16X3G || screened;
  const bool hi_h = prec == YY_PREC_BF16X3G || screened || prec == YY_PREC_BF16X1;
  m.eps_g = split_g ? 0x1p-14 : prec == YY_PREC_BF16X1 ? 0x1p-7 : 0x1p-22;
  m.eps_h = prec == YY_PREC_BF16X3 ? 0x1p-14 : hi_h ? 0x1p-7 : 0x1p-22;
  m.eps_g1 = 0x1p-7;
  for (int s = 0; s < pa.S; ++s) {
    const double kap = ex.kapd[s], tau = ex.taud[s];
    m.kap[s] = (float)kap;
    m.c1[s] = (float)(2.0 * kap);
    // H = X F^T (push) enters with +2 kap tau; H' = F X^T (pull) with -2 kap tau
    m.c2[s] = (float)((pa.pull ? -2.0 : 2.0) * kap * tau);
    m.tau[s] = (float)tau;
    m.kapd[s] = kap;
    m.taud[s] = tau;
  }
  m.bf = pa.bf;
  m.f32t = ex.f32t;
  m.xc = pa.xc;
  m.f = pa.f;
  m.lw2 = pa.lw2;
  m.bsrc = ex.bsrc;
  m.bpre = ex.bpre;
  m.node = pa.node;
  m.bnd = pa.bnd;
  m.scal = pa.scal;
  m.part = pa.part;
  m.nsplit = pa.nsplit;
  m.tb_count = (int)(ex.n_pad / kMI);
  m.group_t = 2;
  m.j_per_split = ex.j_per_split;
  m.flags = ex.flags;
  m.jtl = (pa.n + kMJ - 1) / kMJ;
  m.s_nsplit = pa.nsplit;
  m.s_jps = ((ex.j_per_split + kSJ - 1) / kSJ) * kSJ;
  m.pre_chunks = std::min(kPreK, (int)pa.rp) / kKC;
  m.any_flag = ex.deferred ? ex.deferred->defer : prec == YY_PREC_BF16X3P ? ex.flag_word : nullptr;
  m.rref = pa.pull ? nullptr : ex.rref;
  m.rhv = pa.pull ? nullptr : ex.rhv;
  m.jstar = pa.pull ? nullptr : ex.jstar;
  m.sym_items = ex.sym_items;
  m.tT = ex.tT;
  m.sym_n = ex.sym_n;
  m.sym_list = ex.sym_list;
  m.sym_cap = ex.sym_cap;
  m.sym_nitems = ex.sym_nitems;
  m.ngroups = (int32_t)(ex.n_pad / 64);
  return m;
}

yy_status launch_src_bias(hipStream_t st, const PairArgs& pa, const MfmaExtra& ex) {
  MArgs m = make_args(pa, YY_PREC_BF16X3, ex);
  k_src_bias<<<(unsigned)((ex.n_pad + kBlock - 1) / kBlock), kBlock, 0, st>>>(pa.n, ex.n_pad, pa.S, m, ex.bsrc);
  YY_LAUNCH_CHECK("k_src_bias");
  return YY_OK;
}

yy_status launch_src_bias_heavy(hipStream_t st, const PairArgs& pa, const MfmaExtra& ex, const RowRefArgs& ra) {
  MArgs m = make_args(pa, YY_PREC_BF16X3, ex);
  const int nbias = (int)((ex.n_pad + kBlock - 1) / kBlock);
  k_src_bias_heavy<<<(unsigned)nbias + 1, kBlock, 0, st>>>(pa.n, ex.n_pad, pa.S, m, ex.bsrc, ra, nbias);
  YY_LAUNCH_CHECK("k_src_bias_heavy");
  return YY_OK;
}

template <int S>
static yy_status launch_batch_s(hipStream_t st, const MArgs* sets, const int4* items, int nitems, int prec,
                                bool k64, const BatchScreen* scr) {
  if (prec == YY_PREC_BF16X3) {
    k_pair_mfma_batch<S, 3, 4, 2, false><<<nitems, kNT, 0, st>>>(sets, items);
  } else if (prec == YY_PREC_BF16X3G) {
    k_pair_mfma_batch<S, 2, 4, 2, false><<<nitems, kNT, 0, st>>>(sets, items);
  } else if (prec == YY_PREC_BF16X3S) {
    // four K stages per barrier when every K padding allows it, else two
    if (k64) k_pair_screen_batch<S, 8, 4><<<nitems, kNT, 0, st>>>(sets, items);
    else k_pair_screen_batch<S, 8, 2><<<nitems, kNT, 0, st>>>(sets, items);
    YY_LAUNCH_CHECK("k_pair_mfma_batch (screen)");
    k_pair_mfma_batch<S, 2, 4, 2, true><<<nitems, kNT, 0, st>>>(sets, items);
  } else if (prec == YY_PREC_BF16X3P) {
    // the group bounds of the symmetric sets, the partial-distance screens (symmetric and one-sided
    // items in one launch), the recheck of the doubted units, then the split pass
    if (!scr) return fail(YY_ERR_ARG, "the batched partial-distance screen needs its work lists");
    if (scr->nbound > 0) {
      k_tgt_bound_batch<<<scr->nbound, kBlock, 0, st>>>(sets, scr->bound_items);
      YY_LAUNCH_CHECK("k_tgt_bound_batch");
    }
    if (scr->nscreen > 0) {
      k_pair_prescreen_batch<S><<<scr->nscreen, kPW * 64, 0, st>>>(sets, scr->screen_items);
      YY_LAUNCH_CHECK("k_pair_mfma_batch (partial-distance screen)");
    }
    if (scr->nrecheck > 0) {
      k_sym_recheck_batch<S><<<scr->nrecheck, kPW * 64, 0, st>>>(sets, scr->recheck_items);
      YY_LAUNCH_CHECK("k_sym_recheck_batch");
    }
    k_pair_mfma_batch<S, 2, 4, 2, true><<<nitems, kNT, 0, st>>>(sets, items);
  } else if (prec == YY_PREC_BF16X1) {
    k_pair_mfma_batch<S, 1, 8, 4, false><<<nitems, kNT, 0, st>>>(sets, items);
  } else {
    k_pair_mfma_batch<S, 0, 4, 2, false><<<nitems, kNT, 0, st>>>(sets, items);
  }
  YY_LAUNCH_CHECK("k_pair_mfma_batch");
  return YY_OK;
}

// Pull form: the target side carries the f planes, so the stages are larger
// (BF16X3 40 KB, BF16X3G 32 KB, BF16X1 20 KB, FP32 40 KB) and the rings shorter.
template <int S>
static yy_status launch_pull_s(hipStream_t st, const MArgs& m, int prec, int nblocks) {
  if (prec == YY_PREC_BF16X3) {
    k_pair_mfma<S, 3, 2, 1, false, true><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X3G) {
    k_pair_mfma<S, 2, 4, 2, false, true><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X1) {
    k_pair_mfma<S, 1, 4, 2, false, true><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_FP32_MFMA) {
    k_pair_mfma<S, 0, 2, 1, false, true><<<nblocks, kNT, 0, st>>>(m);
  } else {
    return fail(YY_ERR_UNSUPPORTED, "the pull form has no screened matrix-core form");
  }
  YY_LAUNCH_CHECK("k_pair_mfma (pull form)");
  return YY_OK;
}

template <int S>
static yy_status launch_s(hipStream_t st, const MArgs& m, int prec, int nblocks, const DeferredPrep* dp) {
  if (m.pull) return launch_pull_s<S>(st, m, prec, nblocks);
  if (prec == YY_PREC_BF16X3) {
    k_pair_mfma<S, 3, 4, 2, false><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X3G) {
    k_pair_mfma<S, 2, 4, 2, false><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X3S) {
    // the screen over every tile, then the split form over the flagged tiles
    // four K stages per barrier when the K padding allows it, else two
    if (m.rp % 64 == 0) k_pair_screen<S, 8, 4><<<nblocks, kNT, 0, st>>>(m);
    else k_pair_screen<S, 8, 2><<<nblocks, kNT, 0, st>>>(m);
    YY_LAUNCH_CHECK("k_pair_mfma (screen)");
    k_pair_mfma<S, 2, 4, 2, true><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X3P) {
    // the partial-distance screen (2 or 4 K stages), then the split form over
    // the flagged tiles.  The screen splits the sources only as far as the
    // target blocks leave CUs idle (two blocks per CU): the blocks an XCD runs
    // at a time then stream the same sources through its L2.
    MArgs mp = m;
    int ps = 1;
    const int64_t stiles = (m.n + kPJ - 1) / kPJ;
    while ((int64_t)m.tb_count * ps < 512 && ps < 64 && 2 * ps <= stiles) ps *= 2;
    mp.s_nsplit = ps;
    mp.s_jps = ((stiles + ps - 1) / ps) * kPJ;
    static_assert(kPreK == 64, "4 K stages, or 2 where r_p = 32");
    if (m.sym_items && m.sym_nitems > 0 && m.rref) {
      // many target blocks: the symmetric screen (each pair of target blocks once), after the
      // rows' bounds for its transposed orientation
      k_tgt_bound<<<(unsigned)((m.ngroups + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, st>>>(m);
      YY_LAUNCH_CHECK("k_tgt_bound");
      // (the symmetric screen runs only where the screen spans 64 coordinates: four K stages)
      k_pair_prescreen_sym<S, 4, 16><<<m.sym_nitems, kPW * 64, 0, st>>>(m);
      YY_LAUNCH_CHECK("k_pair_prescreen_sym");
      // the doubted units (a wave each; a grid of two blocks per CU strides over the list)
      k_sym_recheck<S, 4><<<512, kPW * 64, 0, st>>>(m);
    } else if (m.pre_chunks == 4) {
      k_pair_prescreen<S, 4, 16><<<m.tb_count * ps, kPW * 64, 0, st>>>(mp);
    } else {
      k_pair_prescreen<S, 2, 8><<<m.tb_count * ps, kPW * 64, 0, st>>>(mp);
    }
    YY_LAUNCH_CHECK("k_pair_mfma (partial-distance screen)");
    if (dp) {
      // the planes beyond the screen's prefix, if it flagged a tile and they are not yet written
      const yy_status rs = launch_prepare_rest(st, *dp);
      if (rs != YY_OK) return rs;
    }
    k_pair_mfma<S, 2, 4, 2, true><<<nblocks, kNT, 0, st>>>(m);
  } else if (prec == YY_PREC_BF16X1) {
    k_pair_mfma<S, 1, 8, 4, false><<<nblocks, kNT, 0, st>>>(m);
  } else {
    k_pair_mfma<S, 0, 4, 2, false><<<nblocks, kNT, 0, st>>>(m);
  }
  YY_LAUNCH_CHECK("k_pair_mfma");
  return YY_OK;
}

yy_status launch_pair_mfma(hipStream_t st, const PairArgs& pa, int prec, const MfmaExtra& ex) {
  const MArgs m = make_args(pa, prec, ex);
  const int nblocks = m.tb_count * m.nsplit;
  switch (pa.S) {
    case 1: return launch_s<1>(st, m, prec, nblocks, ex.deferred);
    case 2: return launch_s<2>(st, m, prec, nblocks, ex.deferred);
    case 3: return launch_s<3>(st, m, prec, nblocks, ex.deferred);
    case 4: return launch_s<4>(st, m, prec, nblocks, ex.deferred);
  }
  return fail(YY_ERR_UNSUPPORTED, "the matrix-core path supports up to 4 scales");
}

size_t pair_mfma_args_bytes() { return sizeof(MArgs); }

yy_status launch_src_bias_batch(hipStream_t st, const void* sets, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_src_bias_batch<<<total, kBlock, 0, st>>>(static_cast<const MArgs*>(sets), pre, nr);
  YY_LAUNCH_CHECK("k_src_bias_batch");
  return YY_OK;
}

void pair_mfma_fill_args(const PairArgs& pa, int prec, const MfmaExtra& ex, void* out) {
  const MArgs m = make_args(pa, prec, ex);
  std::memcpy(out, &m, sizeof(MArgs));
}

yy_status launch_pair_mfma_batch(hipStream_t st, int S, int prec, const void* sets, const int4* items, int nitems,
                                 bool k64, const BatchScreen* scr) {
  if (nitems <= 0) return YY_OK;
  const MArgs* m = static_cast<const MArgs*>(sets);
  switch (S) {
    case 1: return launch_batch_s<1>(st, m, items, nitems, prec, k64, scr);
    case 2: return launch_batch_s<2>(st, m, items, nitems, prec, k64, scr);
    case 3: return launch_batch_s<3>(st, m, items, nitems, prec, k64, scr);
    case 4: return launch_batch_s<4>(st, m, items, nitems, prec, k64, scr);
  }
  return fail(YY_ERR_UNSUPPORTED, "the matrix-core path supports up to 4 scales");
}

}  // namespace yy
