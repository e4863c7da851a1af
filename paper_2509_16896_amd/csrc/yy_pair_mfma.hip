// yy_pair_mfma.hip -- the pairwise kernel on the CDNA4 matrix cores.
//
// For targets i and sources j (the same node set, centred at the box centre):
//   |x_i - x_j - tau_s f_j|^2 = |x_i|^2 + |m_j^s|^2 - 2 (G_ij + tau_s H_ij),
//   G = X X^T,  H = X F^T,  m_j^s = x_j + tau_s f_j,
// so one pass of two matrix products serves every scale s.  Each block owns
// 256 targets and a range of sources; per 128-source tile it accumulates G and
// H over K = r (zero padded to a multiple of 64) with MFMA 32x32 instructions
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
//   BF16X3: hi/lo split of both operands, hi*hi + lo*hi + hi*lo (3 MFMAs),
//   BF16X1: hi*hi only (a screen),  FP32: v_mfma_f32_32x32x2_f32 on FP32 data.
#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kMI = 256;   // targets per block
constexpr int kMJ = 128;   // sources per tile
constexpr int kKC = 32;    // K per LDS stage
constexpr int kNT = 256;   // 4 waves: 2 along targets x 2 along sources
constexpr int kIB = 4;     // 32-wide target blocks per wave (128 targets)
constexpr int kJB = 2;     // 32-wide source blocks per wave (64 sources)
constexpr float kSkip = 64.f;     // tiles whose exponents are all 2^-64 below the max are skipped

struct MArgs {
  int64_t n, n_pad;
  int32_t r, rp, S;
  float kap[YY_MAX_SCALES];    // log2(e) s / (2 q dt)
  float c1[YY_MAX_SCALES];     // 2 kap_s
  float c2[YY_MAX_SCALES];     // 2 kap_s tau_s
  float tau[YY_MAX_SCALES];
  double kapd[YY_MAX_SCALES];
  double taud[YY_MAX_SCALES];
  const uint16_t* bf;          // bf16 planes [4][rp/32][n_pad][32]: hi(x), hi(f), lo(x), lo(f)
  const float* f32t;           // fp32 planes [2][rp/32][n_pad][32]: x, f
  const float* xc;             // row-major FP32 [n][rp] (exact near pairs)
  const float* f;
  const float* lw2;            // [n]
  const float* bsrc;           // [S][n_pad]: lw2_j - kap_s |m_j^s|^2, -inf for invalid sources
  const double* node;          // [3][n]
  const double* scal;          // [1] = max |x - centre|, [2] = max |f|
  double eps_op;               // relative error of one product from operand rounding
  float2* part;                // [nsplit][S][n]
  int32_t nsplit, tb_count, group_t;
  int64_t j_per_split;
};

// Physical 16-byte chunk of logical chunk c in LDS row `row` (bank-conflict swizzle).
template <int CPR>
__device__ inline int swz(int row, int c) {
  return CPR == 4 ? (c ^ ((row >> 1) & 3)) : (c ^ (row & 7));
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

__device__ inline float exact_pair(const MArgs& a, int64_t i, int64_t j, int s) {
  if (i == j) return a.lw2[j] - (float)(a.kapd[s] * a.taud[s] * a.taud[s] * a.node[a.n + i]);
  const float* xi = a.xc + (size_t)i * a.rp;
  const float* xj = a.xc + (size_t)j * a.rp;
  const float* fj = a.f + (size_t)j * a.rp;
  const float t = a.tau[s];
  float acc = 0.f;
  for (int k = 0; k < a.r; ++k) {
    const float d = xi[k] - xj[k];
    const float e = fmaf(-t, fj[k], d);
    acc = fmaf(e, e, acc);
  }
  return a.lw2[j] - a.kap[s] * acc;
}

// Folds the accumulators of one target (kJB blocks x 16 sources of this lane)
// into the lane's running (max, sum) of that target for every scale.  Flagged
// near pairs are taken out of the approximate set and folded in one at a time
// from their exact values.
__device__ inline void lse2_push(float& M, float& S, float v) {
  if (v == -INFINITY) return;
  if (v > M) {
    S = S * exp2f(M - v) + 1.f;
    M = v;
  } else {
    S += exp2f(v - M);
  }
}

template <int S>
__device__ inline void epilogue_target(const MArgs& a, const f32x16_t (&G)[kJB], const f32x16_t (&H)[kJB],
                                       const float* sb, int64_t i, int64_t j0, int jl0, int g,
                                       const float (&at)[S], const float (&margin)[S], float (&M)[S],
                                       float (&Ssum)[S]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float e[kJB][16];
    float m = -INFINITY;
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int jl = jl0 + jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
        const float base = at[s] + sb[s * kMJ + jl];
        e[jb][v] = fmaf(a.c2[s], H[jb][v], fmaf(a.c1[s], G[jb][v], base));
        m = fmaxf(m, e[jb][v]);
      }
    if (!(m > M[s] - kSkip)) continue;
    const float thr = fmaxf(M[s], m) - margin[s];
    uint32_t flagged = 0u;
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        if (e[jb][v] >= thr) {
          flagged |= 1u << (jb * 16 + v);
          e[jb][v] = -INFINITY;
        }
    while (flagged) {
      const int bit = __builtin_ctz(flagged);
      flagged &= flagged - 1u;
      const int jb = bit >> 4, v = bit & 15;
      const int jl = jl0 + jb * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
      lse2_push(M[s], Ssum[s], exact_pair(a, i, j0 + jl, s));
    }
    float m2 = -INFINITY;
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v) m2 = fmaxf(m2, e[jb][v]);
    const float Mn = fmaxf(M[s], m2);
    if (Mn == -INFINITY) continue;
    float sum = Ssum[s] * exp2f(M[s] - Mn);
#pragma unroll
    for (int jb = 0; jb < kJB; ++jb)
#pragma unroll
      for (int v = 0; v < 16; ++v) sum += exp2f(e[jb][v] - Mn);
    Ssum[s] = sum;
    M[s] = Mn;
  }
}

// Final merge: lanes l and l^32 hold the same target; waves (wi, 0) and
// (wi, 1) hold the same targets.  Writes part[split][s][i].
template <int S>
__device__ inline void merge_and_store(const MArgs& a, float (&M)[kIB][S], float (&Ssum)[kIB][S],
                                       int64_t i0, int split, float2* xchg) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1, col = lane & 31, g = lane >> 5;
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float mo = __shfl_xor(M[ib][s], 32, 64);
      const float so = __shfl_xor(Ssum[ib][s], 32, 64);
      lse2_merge(M[ib][s], Ssum[ib][s], mo, so);
    }
  __syncthreads();
  if (wj == 1 && g == 0) {
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
      for (int s = 0; s < S; ++s)
        xchg[((wi * kIB + ib) * 32 + col) * S + s] = make_float2(M[ib][s], Ssum[ib][s]);
  }
  __syncthreads();
  if (wj == 0 && g == 0) {
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float2 o = xchg[((wi * kIB + ib) * 32 + col) * S + s];
        lse2_merge(M[ib][s], Ssum[ib][s], o.x, o.y);
        if (i < a.n) a.part[((size_t)split * S + s) * a.n + i] = make_float2(M[ib][s], Ssum[ib][s]);
      }
    }
  }
}

// Rigorous bound on |e_approx - e_exact| in base-2 units: operand rounding,
// worst-case FP32 accumulation over rp products, FP32 evaluation of e; the
// margin adds the skip depth and 16 bits of safety.
template <int S>
__device__ inline void init_targets(const MArgs& a, int64_t i0, float (&at)[kIB][S], float (&M)[kIB][S],
                                    float (&Ssum)[kIB][S], float (&margin)[S]) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, col = lane & 31;
  const double X = a.scal[1], F = a.scal[2];
  const double gam = a.rp * 0x1p-24;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double XT = X + a.taud[s] * F;
    const double dD = (a.eps_op + gam) * 2.0 * X * XT + 16.0 * 0x1p-24 * XT * XT;
    margin[s] = (float)(2.0 * a.kapd[s] * dD + (double)kSkip + 16.0);
  }
#pragma unroll
  for (int ib = 0; ib < kIB; ++ib) {
    const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
    const double nx = i < a.n ? a.node[i] : 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      at[ib][s] = i < a.n ? (float)(-a.kapd[s] * nx) : -INFINITY;
      M[ib][s] = -INFINITY;
      Ssum[ib][s] = 0.f;
    }
  }
}

// Direct global -> LDS copy of one K stage (global_load_lds_dwordx4): each
// instruction moves 1 KB, lane L landing at byte 16 L of the region, so the
// bank-conflict swizzle is applied by choosing which global chunk a lane loads.
// ROWB = bytes per row per stage (64: bf16 planes, 128: fp32 planes).
template <int ROWB, int NTP, int NSP>
__device__ inline void issue_stage(const MArgs& a, const void* const* tplane, const void* const* splane,
                                   unsigned char* stage, int c, int64_t i0, int64_t j0) {
  constexpr int CPR = ROWB / 16;               // 16-byte chunks per row
  constexpr int RPR = 64 / CPR;                // rows per 1 KB region
  constexpr int TREG = kMI / RPR, SREG = kMJ / RPR;
  constexpr int R = NTP * TREG + NSP * SREG;
  constexpr int ESZ = ROWB / kKC;              // element size in bytes
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rl = lane / CPR, pc = lane % CPR;
#pragma unroll
  for (int u = 0; u < R / 4; ++u) {
    const int q = wave + 4 * u;
    const unsigned char* src;
    int off;
    if (q < NTP * TREG) {
      const int p = q / TREG, rb = (q % TREG) * RPR, row = rb + rl;
      const int lc = swz<CPR>(row, pc);
      src = static_cast<const unsigned char*>(tplane[p]) +
            (((size_t)c * a.n_pad + (size_t)(i0 + row)) * kKC) * ESZ + lc * 16;
      off = p * (kMI * ROWB) + rb * ROWB;
    } else {
      const int q2 = q - NTP * TREG;
      const int p = q2 / SREG, rb = (q2 % SREG) * RPR, row = rb + rl;
      const int lc = swz<CPR>(row, pc);
      src = static_cast<const unsigned char*>(splane[p]) +
            (((size_t)c * a.n_pad + (size_t)(j0 + row)) * kKC) * ESZ + lc * 16;
      off = NTP * kMI * ROWB + p * (kMJ * ROWB) + rb * ROWB;
    }
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                     (__attribute__((address_space(3))) void*)(stage + off), 16, 0, 0);
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

// ---------------------------------------------------------------------------
// BF16 variants.  LDS stage: target planes [NTP][256 rows][64 B] (hi, lo of x),
// source planes [NSP][128 rows][64 B] (hi x, hi f, lo x, lo f); NTP = 2, NSP = 4
// for the hi/lo split, 1 and 2 for hi only.  Each wave: 128 targets x 64 sources.
template <int S, int PASSES>
__global__ void __launch_bounds__(kNT, 1) k_pair_mfma_bf16(MArgs a) {
  constexpr int NTP = PASSES == 3 ? 2 : 1;
  constexpr int NSP = PASSES == 3 ? 4 : 2;
  constexpr int ROWB = 64;
  constexpr int TB = NTP * kMI * ROWB;
  constexpr int STAGE = TB + NSP * kMJ * ROWB;
  __shared__ __attribute__((aligned(1024))) unsigned char smem[2 * STAGE];
  __shared__ float sb[YY_MAX_SCALES * kMJ];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1, col = lane & 31, g = lane >> 5;
  int tb, split;
  block_map(a, tb, split);
  const int64_t i0 = (int64_t)tb * kMI;
  const int64_t jb0 = (int64_t)split * a.j_per_split;
  const int64_t jb1 = jb0 + a.j_per_split < a.n ? jb0 + a.j_per_split : a.n;
  const int nchunks = a.rp / kKC;
  const size_t plane = (size_t)nchunks * a.n_pad * kKC;   // elements per global plane
  const void* sp[4] = {a.bf, a.bf + plane, a.bf + 2 * plane, a.bf + 3 * plane};
  const void* tp[2] = {a.bf, a.bf + 2 * plane};

  float at[kIB][S], M[kIB][S], Ssum[kIB][S], margin[S];
  init_targets<S>(a, i0, at, M, Ssum, margin);

  for (int64_t j0 = jb0; j0 < jb1; j0 += kMJ) {
    f32x16_t G[kIB][kJB], H[kIB][kJB];
    zero_acc<S>(G, H);
    __syncthreads();   // the previous tile's readers are done with stage 0 and sb
    issue_stage<ROWB, NTP, NSP>(a, tp, sp, smem, 0, i0, j0);
    for (int t = tid; t < S * kMJ; t += kNT) sb[t] = a.bsrc[(size_t)(t / kMJ) * a.n_pad + j0 + (t % kMJ)];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int c = 0; c < nchunks; ++c) {
      const int stage = c & 1;
      if (c + 1 < nchunks) issue_stage<ROWB, NTP, NSP>(a, tp, sp, smem + (stage ^ 1) * STAGE, c + 1, i0, j0);
      const unsigned char* base = smem + stage * STAGE;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int lc = 2 * ks + g;   // logical 16-byte chunk of this lane group
        bf16x8_t bh[kIB], bl[kIB], xh[kJB], xl[kJB], fh[kJB], fl[kJB];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) {
          const int row = wi * (32 * kIB) + ib * 32 + col;
          const int off = row * ROWB + swz<4>(row, lc) * 16;
          bh[ib] = *reinterpret_cast<const bf16x8_t*>(base + off);
          if (PASSES == 3) bl[ib] = *reinterpret_cast<const bf16x8_t*>(base + kMI * ROWB + off);
        }
#pragma unroll
        for (int jb = 0; jb < kJB; ++jb) {
          const int row = wj * (32 * kJB) + jb * 32 + col;
          const int off = TB + row * ROWB + swz<4>(row, lc) * 16;
          xh[jb] = *reinterpret_cast<const bf16x8_t*>(base + off);
          fh[jb] = *reinterpret_cast<const bf16x8_t*>(base + kMJ * ROWB + off);
          if (PASSES == 3) {
            xl[jb] = *reinterpret_cast<const bf16x8_t*>(base + 2 * kMJ * ROWB + off);
            fl[jb] = *reinterpret_cast<const bf16x8_t*>(base + 3 * kMJ * ROWB + off);
          }
        }
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
          for (int jb = 0; jb < kJB; ++jb) {
            G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bh[ib], G[ib][jb], 0, 0, 0);
            H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[jb], bh[ib], H[ib][jb], 0, 0, 0);
            if (PASSES == 3) {
              G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[jb], bh[ib], G[ib][jb], 0, 0, 0);
              H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl[jb], bh[ib], H[ib][jb], 0, 0, 0);
              G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[jb], bl[ib], G[ib][jb], 0, 0, 0);
              H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[jb], bl[ib], H[ib][jb], 0, 0, 0);
            }
          }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
      epilogue_target<S>(a, G[ib], H[ib], sb, i, j0, wj * (32 * kJB), g, at[ib], margin, M[ib], Ssum[ib]);
    }
  }
  merge_and_store<S>(a, M, Ssum, i0, split, reinterpret_cast<float2*>(smem));
}

// ---------------------------------------------------------------------------
// FP32 variant (v_mfma_f32_32x32x2_f32).  LDS stage: target plane [256 rows][128 B],
// source planes x, f [128 rows][128 B].  Within a 32-wide K stage, lane group g
// owns k = 16 g + t in K step t (any fixed assignment of k to steps is valid as
// long as both operands use it), so each lane reads 16 consecutive floats.
template <int S>
__global__ void __launch_bounds__(kNT, 1) k_pair_mfma_f32(MArgs a) {
  constexpr int ROWB = 128;
  constexpr int TB = kMI * ROWB;
  constexpr int STAGE = TB + 2 * kMJ * ROWB;
  __shared__ __attribute__((aligned(1024))) unsigned char smem[2 * STAGE];
  __shared__ float sb[YY_MAX_SCALES * kMJ];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1, col = lane & 31, g = lane >> 5;
  int tb, split;
  block_map(a, tb, split);
  const int64_t i0 = (int64_t)tb * kMI;
  const int64_t jb0 = (int64_t)split * a.j_per_split;
  const int64_t jb1 = jb0 + a.j_per_split < a.n ? jb0 + a.j_per_split : a.n;
  const int nchunks = a.rp / kKC;
  const size_t plane = (size_t)nchunks * a.n_pad * kKC;
  const void* sp[2] = {a.f32t, a.f32t + plane};
  const void* tp[1] = {a.f32t};

  float at[kIB][S], M[kIB][S], Ssum[kIB][S], margin[S];
  init_targets<S>(a, i0, at, M, Ssum, margin);

  for (int64_t j0 = jb0; j0 < jb1; j0 += kMJ) {
    f32x16_t G[kIB][kJB], H[kIB][kJB];
    zero_acc<S>(G, H);
    __syncthreads();
    issue_stage<ROWB, 1, 2>(a, tp, sp, smem, 0, i0, j0);
    for (int t = tid; t < S * kMJ; t += kNT) sb[t] = a.bsrc[(size_t)(t / kMJ) * a.n_pad + j0 + (t % kMJ)];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int c = 0; c < nchunks; ++c) {
      const int stage = c & 1;
      if (c + 1 < nchunks) issue_stage<ROWB, 1, 2>(a, tp, sp, smem + (stage ^ 1) * STAGE, c + 1, i0, j0);
      const unsigned char* base = smem + stage * STAGE;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int lc = 4 * g + u;
        float4 bt[kIB], xs[kJB], fs[kJB];
#pragma unroll
        for (int ib = 0; ib < kIB; ++ib) {
          const int row = wi * (32 * kIB) + ib * 32 + col;
          bt[ib] = *reinterpret_cast<const float4*>(base + row * ROWB + swz<8>(row, lc) * 16);
        }
#pragma unroll
        for (int jb = 0; jb < kJB; ++jb) {
          const int row = wj * (32 * kJB) + jb * 32 + col;
          const int off = TB + row * ROWB + swz<8>(row, lc) * 16;
          xs[jb] = *reinterpret_cast<const float4*>(base + off);
          fs[jb] = *reinterpret_cast<const float4*>(base + kMJ * ROWB + off);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int ib = 0; ib < kIB; ++ib)
#pragma unroll
            for (int jb = 0; jb < kJB; ++jb) {
              G[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[jb][e], bt[ib][e], G[ib][jb], 0, 0, 0);
              H[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(fs[jb][e], bt[ib][e], H[ib][jb], 0, 0, 0);
            }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
#pragma unroll
    for (int ib = 0; ib < kIB; ++ib) {
      const int64_t i = i0 + wi * (32 * kIB) + ib * 32 + col;
      epilogue_target<S>(a, G[ib], H[ib], sb, i, j0, wj * (32 * kJB), g, at[ib], margin, M[ib], Ssum[ib]);
    }
  }
  merge_and_store<S>(a, M, Ssum, i0, split, reinterpret_cast<float2*>(smem));
}

// ---------------------------------------------------------------------------
// Source biases b_js = lw2_j - kap_s |m_j^s|^2 (FP64 -> FP32), -inf for invalid sources.
__global__ void __launch_bounds__(kBlock) k_src_bias(int64_t n, int64_t n_pad, int32_t S,
                                                     MArgs a, float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n_pad) return;
  for (int s = 0; s < S; ++s) {
    float v = -INFINITY;
    if (j < n) {
      const float l = a.lw2[j];
      if (l != -INFINITY) {
        const double t = a.taud[s];
        const double nm = a.node[j] + 2.0 * t * a.node[2 * n + j] + t * t * a.node[n + j];
        v = (float)((double)l - a.kapd[s] * nm);
      }
    }
    out[(size_t)s * n_pad + j] = v;
  }
}

int64_t pair_mfma_npad(int64_t n) { return ((n + kMI - 1) / kMI) * kMI; }

static MArgs make_args(const PairArgs& pa, int prec, const MfmaExtra& ex) {
  MArgs m{};
  m.n = pa.n;
  m.n_pad = ex.n_pad;
  m.r = pa.r;
  m.rp = pa.rp;
  m.S = pa.S;
  m.eps_op = prec == YY_PREC_BF16X3 ? 0x1p-14 : prec == YY_PREC_BF16X1 ? 0x1p-7 : 0x1p-22;
  for (int s = 0; s < pa.S; ++s) {
    const double kap = ex.kapd[s], tau = ex.taud[s];
    m.kap[s] = (float)kap;
    m.c1[s] = (float)(2.0 * kap);
    m.c2[s] = (float)(2.0 * kap * tau);
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
  m.node = pa.node;
  m.scal = pa.scal;
  m.part = pa.part;
  m.nsplit = pa.nsplit;
  m.tb_count = (int)(ex.n_pad / kMI);
  m.group_t = 2;
  m.j_per_split = ex.j_per_split;
  return m;
}

yy_status launch_src_bias(hipStream_t st, const PairArgs& pa, const MfmaExtra& ex) {
  MArgs m = make_args(pa, YY_PREC_BF16X3, ex);
  k_src_bias<<<(unsigned)((ex.n_pad + kBlock - 1) / kBlock), kBlock, 0, st>>>(pa.n, ex.n_pad, pa.S, m, ex.bsrc);
  YY_LAUNCH_CHECK("k_src_bias");
  return YY_OK;
}

template <int S>
static yy_status launch_s(hipStream_t st, const MArgs& m, int prec, int nblocks) {
  if (prec == YY_PREC_BF16X3) k_pair_mfma_bf16<S, 3><<<nblocks, kNT, 0, st>>>(m);
  else if (prec == YY_PREC_BF16X1) k_pair_mfma_bf16<S, 1><<<nblocks, kNT, 0, st>>>(m);
  else k_pair_mfma_f32<S><<<nblocks, kNT, 0, st>>>(m);
  YY_LAUNCH_CHECK("k_pair_mfma");
  return YY_OK;
}

yy_status launch_pair_mfma(hipStream_t st, const PairArgs& pa, int prec, const MfmaExtra& ex) {
  const MArgs m = make_args(pa, prec, ex);
  const int nblocks = m.tb_count * m.nsplit;
  switch (pa.S) {
    case 1: return launch_s<1>(st, m, prec, nblocks);
    case 2: return launch_s<2>(st, m, prec, nblocks);
    case 3: return launch_s<3>(st, m, prec, nblocks);
    case 4: return launch_s<4>(st, m, prec, nblocks);
  }
  return fail(YY_ERR_UNSUPPORTED, "the matrix-core path supports up to 4 scales");
}

}  // namespace yy
