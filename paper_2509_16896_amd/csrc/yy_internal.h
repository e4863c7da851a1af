// yy_internal.h -- shared declarations of libyy's host and device code (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#include <string>
#include <vector>

#include "../../include/yy.h"

namespace yy {

constexpr int kBlock = 256;          // threads per block of the support kernels
constexpr int kWave = 64;            // CDNA wavefront width
constexpr double kBoundaryTol = 1e-12;  // distance to a face that marks a boundary node
constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr double kLn2 = 0.69314718055994530941723212145818;
constexpr int kPreK = 64;             // coordinates of the partial-distance screen (BF16X3P)
constexpr double kNoisePinvRtol = 1e-10;  // eigenvalues of a, b at or below this fraction of the largest are zero
constexpr int32_t kDriftGiven = 100;  // internal drift code: f(x) read from a precomputed array

// Sets the thread-local error text and returns `st`.
yy_status fail(yy_status st, const std::string& msg);
yy_status hip_fail(hipError_t e, const char* what);

#define YY_HIP(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::yy::hip_fail(e_, #call); \
  } while (0)

#define YY_LAUNCH_CHECK(name)                                   \
  do {                                                          \
    hipError_t e_ = hipGetLastError();                          \
    if (e_ != hipSuccess) return ::yy::hip_fail(e_, name);      \
  } while (0)

// Grow-only device buffer owned by the context.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  yy_status ensure(size_t want);
  void release();
  template <class T>
  T* as() const { return static_cast<T*>(ptr); }
};

// The node set as the pairwise kernels consume it; rebuilt when the nodes change.
// BF16X3P on one run: the preparation writes only what the partial-distance
// screen reads (the node norms, the boundary flags and hi(xc) over the first
// kPreK coordinates); the remaining planes are written after the screen, and
// only once it has flagged a tile for this node set.
struct DeferredPrep {
  int64_t n, n_pad;
  int32_t r, rp, drift;
  const double *A, *x, *lo, *hi;
  float *xc32, *f32;
  uint16_t* bf;
  int* defer;   // device int[2]: [0] the screen flagged a tile in this call, [1] the planes are complete
};
yy_status launch_prepare_rest(hipStream_t st, const DeferredPrep& d);

struct Prepared {
  bool valid = false;
  bool deferred = false;    // the planes beyond the screen's prefix wait for a flagged tile (dp)
  DeferredPrep dp{};
  const double* x = nullptr;
  int64_t n = 0;
  int32_t r = 0;
  int32_t rp = 0;           // r rounded up to the matrix-core K step (zero padded)
  int32_t drift = -1;
  const double* A = nullptr;
  uint64_t version = 0;
  const double* lo = nullptr;
  const double* hi = nullptr;
  bool have_bf16 = false;
  bool have_f32t = false;
  int64_t n_pad = 0;        // n rounded up to the matrix-core target block
  DevBuf xc32;              // float [n*rp]  x - box centre
  DevBuf f32;               // float [n*rp]  f(x)
  DevBuf bf;                // bf16 tiled [4][rp/16][n_pad][16]: hi(xc), hi(f), lo(xc), lo(f)
  DevBuf f32t;              // float tiled [2][rp/16][n_pad][16]: xc, f
  DevBuf node;              // double [6][n]  |xc|^2, |f|^2, xc.f, the same over the first kPreK
                            // coordinates; then 4 maxima per preparation block
  DevBuf bnd;               // int [n]  1 = boundary node
  DevBuf scal;              // double [6]  log vol(box), max |xc|, max |f|, spare, the maxima over kPreK
  DevBuf div;               // double [n]  div f(x_i) (pull form), valid for (version, div_mode)
  int32_t div_mode = -1;    // the divergence computed in div, -1: none
  // general process noise: centred nodes and drift values in the original coordinates, then
  // their whitened images W x, W f (the pairwise kernels' inputs), and the boundary flags
  DevBuf wtmp;              // double [2][n][r]
  DevBuf wnodes;            // double [2][n][k]
  DevBuf wbnd;              // int [n]
  const void* noise = nullptr;
};

// Whitened node set of a model with general process noise (noise_whiten_nodes).
struct WhiteNodes {
  const double* x;      // [n][k]  W (x - centre)
  const double* f;      // [n][k]  W f(x)
  const int* bnd;       // [n]     boundary flags from the original coordinates and box
  const double* zeros;  // [>= k]  zero vector (the whitened box centre)
  int32_t k;
};

}  // namespace yy

struct yy_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  uint32_t* d_flags = nullptr;        // status word
  unsigned long long* d_nclamped = nullptr;
  int* d_defer = nullptr;             // int[2] of the deferred planes (DeferredPrep::defer)
  // Sobol direction numbers (host, unscrambled) for dimensions < dir_r.
  std::vector<uint32_t> dirs;
  int32_t dir_r = 0;
  yy::DevBuf d_dirs;                  // uint32 [r][33]: 32 scrambled direction numbers + shift
  int32_t d_dirs_r = -1;
  int32_t d_dirs_scramble = -1;
  uint64_t d_dirs_seed = 0;
  yy::Prepared prep;
  yy::DevBuf lw2;                     // float [n]: source log2-weights relative to their max
  yy::DevBuf part;                    // pairwise partial (max, sum) results
  yy::DevBuf red;                     // reduction scratch
  yy::DevBuf red2;
  yy::DevBuf scan;                    // resampling prefix sums
  yy::DevBuf bsrc;                    // matrix-core source biases
  yy::DevBuf sflags;                  // screen verdicts of the screened split form
  yy::DevBuf obsw;                    // general observation noise: h(x) rows, W_b h(x) rows, W_b dy
  yy::DevBuf rref;                    // float [2][S][n]: lower bounds of the pairwise rows' maxima, heavy-pair terms
  yy::DevBuf sym_items, tT, sym_list;  // the symmetric screen: int4 work items; float [2][S][n_pad / 64];
                                       // the doubted units' counter (16 bytes) and int4 list
  int64_t sym_tbs = 0;                // target blocks the items were built for
  int sym_nitems = 0;
  int sym_cap = 0;                    // list entries: 8 per tile of the items (2 row groups x 4 waves), at most kSymListMax
  yy::DevBuf fstar;                   // double [r]: f at the heaviest source
  int64_t sflags_tbs = 0, sflags_jtl = 0;   // their shape at the last screened propagation
  // tuned source-split counts: (rp, n_pad, S, prec) -> nsplit
  struct TuneEntry {
    int32_t rp;
    int64_t n_pad;
    int32_t S, prec, nsplit;
  };
  std::vector<TuneEntry> tune;
  // pairwise-kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_used = 0;
};

// General noise coefficients (yy_noise.hip): whitening rows W_a (rank_a x r)
// and W_b (rank_b x m) with W^T W the pseudo-inverse, and log det_+.
struct yy_noise_s {
  yy_ctx ctx = nullptr;
  int32_t r = 0, m = 0;
  int32_t rank_a = 0, rank_b = 0;   // 0: isotropic (q I, rho2 I from the model)
  double logdet_a = 0.0, logdet_b = 0.0;
  yy::DevBuf Wa, Wb, zeros;
};

// The learned restart proposal's state (yy_proposal.hip).
struct yy_proposal_s {
  yy_ctx ctx = nullptr;
  int32_t r = 0, H = 0;
  int64_t P = 0;
  yy::DevBuf params, adam_m, adam_v, grad, work, part;
  int64_t work_B = 0;
  int64_t t = 0;   // Adam steps taken
  // offsets of W1, b1, W2, b2, W3, b3 in the parameter vector
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float* pf() const { return params.as<float>(); }
};

namespace yy {

// Host-side pieces shared by the call implementations.
yy_status sobol_prepare_dirs(yy_ctx ctx, int32_t r, int32_t scramble, uint64_t seed);
yy_status prepare_nodes(yy_ctx ctx, const yy_model* model, int64_t n, const double* x,
                        uint64_t version, const double* lo, const double* hi, bool want_bf16,
                        bool want_f32t, int32_t prec, bool defer_planes);
yy_status coefficients_cramer(int32_t S, const double* s, double* c);
yy_status validate_model(const yy_model* m);
yy_status timing_begin(yy_ctx ctx);
yy_status timing_end(yy_ctx ctx);
// Locates the no-allocation scratch of the current device (yy_update.hip); called by yy_create.
yy_status noalloc_scratch_init(int device);
// General noise (yy_noise.hip): the whitened node set, and the correction with b^+.
yy_status noise_whiten_nodes(yy_ctx ctx, const yy_model* m, int64_t n, const double* x, const double* lo,
                             const double* hi, WhiteNodes& out);
yy_status noise_loglik(yy_ctx ctx, const yy_model* m, int64_t n, const double* x, const double* dy, double dt,
                       double* logw);
inline bool noise_a(const yy_model* m) { return m->noise && m->noise->rank_a > 0; }
inline bool noise_b(const yy_model* m) { return m->noise && m->noise->rank_b > 0; }

// Pairwise kernel launchers (per-(target, scale) partial max/sum in base 2).
struct PairArgs {
  int64_t n;
  int32_t r, rp, S;
  float kap2[YY_MAX_SCALES];   // log2(e) * s / (2 q dt): multiplies |x_i - m_j|^2
  float tau[YY_MAX_SCALES];    // dt / s
  const float* xc;
  const float* f;
  const float* lw2;            // [n]
  const double* node;          // [3][n]
  const int* bnd;
  const uint16_t* bf;          // [4][n*rp] or null
  const double* scal;
  float2* part;                // [nsplit][S][n]
  int32_t nsplit;
  int32_t pull;                // pull-form kernel (eq. kernel) instead of the push form
};
// Extra inputs of the matrix-core kernel.
struct MfmaExtra {
  int64_t n_pad;               // rows of the tiled planes (n rounded up to the target block)
  const float* f32t;           // fp32 tiled planes (FP32 variant) or null
  float* bsrc;                 // [S][n_pad] source biases (written by launch_src_bias)
  int64_t j_per_split;
  double kapd[YY_MAX_SCALES];
  double taud[YY_MAX_SCALES];
  uint8_t* flags;              // screened split forms: [n_pad/256][ceil(n/128)][8] screen verdicts
  float* bpre;                 // BF16X3P: source biases over the first kPreK coordinates, laid out as bsrc
  const DeferredPrep* deferred;   // BF16X3P on one run with deferred planes, else null
  // BF16X3P without deferred planes (the batched step): a device word that the source biases clear and
  // the screens raise when they flag a tile, so that with none flagged the split pass writes nothing
  // and the combination forms the self-pair splits' states (null: every split written and combined)
  int* flag_word = nullptr;
  const float* rref = nullptr;     // [S][n] lower bounds of the row maxima (push form), or null: self pairs
  const float* rhv = nullptr;      // [S][n] the pair (i, j*) counted apart (exact term), or -inf; with rref
  const long long* jstar = nullptr;   // j*, the heaviest source (-1: none); with rref
  // BF16X3P on one run with more than kSymMinBlocks target blocks: the symmetric screen's work items
  // (A, B0, B1), its row bounds ([2][S][n_pad / 64] per 64-row group), and the counter and list of the
  // units whose coarse bound doubted (room for sym_cap)
  const int4* sym_items = nullptr;
  float* tT = nullptr;
  int sym_nitems = 0;
  int* sym_n = nullptr;
  int4* sym_list = nullptr;
  int sym_cap = 0;
};
constexpr int kSymMinBlocks = 32;   // target blocks of 256 above which the symmetric screen runs (r_p > 32)
constexpr int64_t kSymListMax = 1 << 20;   // doubted units held at most (a full list flags the rest)
constexpr int kSymChunk = 32;       // target blocks of sources per work item
// The symmetric screen's work items for tbs target blocks: (A, B0, B1, 0), target block A against the
// target blocks [B0, B1) >= A as sources, kSymChunk at a time, the longest first (then by source range,
// so that items started together share sources).
std::vector<int4> sym_work_items(int64_t tbs);
// blocks of the node preparation kernel (one wave per 4 nodes, grid-stride)
// Node preparation takes a wavefront per node up to kPrepWideMax padded nodes (a short
// chain of steps per row where the node set is small), 16 lanes per node beyond.
constexpr int64_t kPrepWideMax = 8192;
__host__ __device__ inline bool prep_wide(int64_t n_pad) { return n_pad <= kPrepWideMax; }
int prepare_blocks(int64_t n_pad);
yy_status launch_src_bias(hipStream_t st, const PairArgs& a, const MfmaExtra& ex);
yy_status launch_pair_mfma(hipStream_t st, const PairArgs& a, int prec, const MfmaExtra& ex);
// Batched matrix-core kernel: `sets` is a device array of the per-set kernel
// arguments (pair_mfma_args_bytes() each, filled by pair_mfma_fill_args);
// items[b] = (set, target block, source split, cost).
size_t pair_mfma_args_bytes();
void pair_mfma_fill_args(const PairArgs& pa, int prec, const MfmaExtra& ex, void* out);
// k64: every set's K padding is a multiple of 64 (the screen's four-stage groups).
// BF16X3P takes its screen's work lists (device int4 arrays) in `scr`: the screen items, (set, A, B0,
// B1) of the symmetric screen for sets of more than kSymMinBlocks target blocks, (set, target block,
// source split, -1) for the others; the group-bound items (set, block, 0, 0) and the recheck items
// (set, block, blocks of the set, 0) of the symmetric sets.
struct BatchScreen {
  const int4* screen_items = nullptr;
  int nscreen = 0;
  const int4* bound_items = nullptr;
  int nbound = 0;
  const int4* recheck_items = nullptr;
  int nrecheck = 0;
};
yy_status launch_pair_mfma_batch(hipStream_t st, int S, int prec, const void* sets, const int4* items, int nitems,
                                 bool k64, const BatchScreen* scr = nullptr);

// (4) combination in FP64: merge the source splits, add the constants, signed
// log-sum-exp over the scales and the identity term.
// The state (maximum, sum; base 2) with which target i's partial sum at scale s
// starts in the source split that holds its self pair: the row floor rref as the
// maximum (the self-pair exponent where there is none), and in the sum the self
// pair's term and, where the row counts it apart, the heavy pair's exact term rhv.
// li: the target's source weight (lw2); fnorm: |f(x_i)|^2.  The other splits
// start at (maximum, 0).  A split whose source range holds no flagged tile keeps
// this state; where a call flags no tile at all, the combination forms it here
// rather than reading it from the split form's output.
__device__ __forceinline__ float2 owner_start(float li, double fnorm, double kapd, double taud, const float* rref,
                                              const float* rhv, int64_t n, int64_t i, int s) {
  const float self = li != -INFINITY ? li - (float)(kapd * taud * taud * fnorm) : -INFINITY;
  const float M0 = rref ? rref[(size_t)s * n + i] : self;
  const float h = rhv ? rhv[(size_t)s * n + i] : -INFINITY;
  float sum = self != -INFINITY ? (self == M0 ? 1.f : __builtin_amdgcn_exp2f(self - M0)) : 0.f;
  if (h != -INFINITY) sum += h == M0 ? 1.f : __builtin_amdgcn_exp2f(h - M0);
  return make_float2(M0, sum);
}

struct CombineArgs {
  int64_t n;
  int32_t S, nsplit;
  double kap[YY_MAX_SCALES];       // log|c_s| - log n - (r/2) log(2 pi q tau_s)
  double sign[YY_MAX_SCALES + 1];  // sign(c_s), 0 for c_s = 0
  double logc_id;                  // log|c_S|
  const float2* part;
  const double* scal;              // [0] = log vol(box)
  const double* lref;              // max source log-weight
  const double* logw_in;
  const int* bnd;
  double* logw_out;
  uint32_t* flags;
  unsigned long long* nclamped;
  int* defer;                      // deferred planes: marked complete when the screen flagged a tile
  int64_t j_per_split;             // sources per split of the matrix-core kernel
  const double* div;               // pull form: div f(x_i) [n]; its factor exp(-tau_s div) per scale, else null
  double taud[YY_MAX_SCALES];      // tau_s
  // the self-pair split's starting state (owner_start) where no tile of the call is flagged (defer[0] = 0)
  double kapd[YY_MAX_SCALES];      // the pairwise kernel's kappa_s
  const float* lw2;                // source weights [n]
  const double* node;              // node norms ([n, 2n) holds |f|^2)
  const float* rref;               // row floors [S][n], or null
  const float* rhv;                // heavy-pair terms [S][n], or null
};

// One yy_propagate call split into its phases: begin = node preparation,
// source weights, biases and the launch parameters; pair = the pairwise
// kernel; end = the combination.  nsplit_override > 0 fixes the number of
// source splits of the matrix-core kernel.
// One node set of the batched vector-ALU pairwise launch: its arguments, source range per split and
// FP64 scale constants, as the single-run launch passes them.
struct ValuSet {
  PairArgs a;
  int64_t per;
  double taud[YY_MAX_SCALES], kapd[YY_MAX_SCALES];
};
int valu_kc(int32_t r);                  // coordinates staged per step: 2, 4, 8 or 16
int64_t valu_per(const PairArgs& a);     // sources per split
yy_status launch_pair_valu_batch(hipStream_t st, int32_t S, int kc, const ValuSet* sets, const int4* items,
                                 int nitems);

struct PropPlan {
  int64_t n = 0;
  int32_t prec = 0;
  bool mfma = false;
  PairArgs a{};
  MfmaExtra ex{};
  CombineArgs cb{};
  double taud[YY_MAX_SCALES] = {0, 0, 0, 0, 0, 0};
  double kapd[YY_MAX_SCALES] = {0, 0, 0, 0, 0, 0};
};
yy_status propagate_begin(yy_ctx ctx, const yy_model* model, const yy_scales* scales, int32_t prec, int64_t n,
                          const double* x, uint64_t node_version, const double* box_lo, const double* box_hi,
                          double dt, const double* logw_in, double* logw_out, int nsplit_override,
                          PropPlan& plan, bool defer_planes = false);
yy_status propagate_pair(yy_ctx ctx, const PropPlan& plan);
yy_status propagate_end(yy_ctx ctx, const PropPlan& plan);
// Step (2) alone (lw2 and the device address of the weights' maximum, in ctx->red) and step (4)'s launch.
yy_status source_weights(yy_ctx ctx, int64_t n, const double* logw_in, const int* bnd, float* lw2,
                         double** lref_out, long long** heavy_out = nullptr);
yy_status launch_combine(hipStream_t st, const CombineArgs& cb);

// Blocks of the normalisation kernels for n nodes: 64 rows per block (at most 1024
// blocks), enough blocks to stream the n x r coordinates at full bandwidth; up to
// n = 4096, 16 rows per block, so that a wave's chain of rows is short where the
// kernel is bound by latency rather than bandwidth.
constexpr int kMaxNormBlocks = 1024;   // the largest norm_blocks(n)
inline int norm_blocks(int64_t n) {
  if (n <= 4096) return (int)((n + 15) / 16);
  return (int)((n + 63) / 64 < 1024 ? (n + 63) / 64 : 1024);
}

// Targets per block of the row-floor kernel: 16 rows of 16 lanes each where r <= 256;
// for longer rows the whole wave across a row's coordinates, one row per wave up to
// n = 8192 (latency-bound sizes), four rows per wave beyond.
__host__ __device__ inline int row_ref_targets(int32_t r, int64_t n) { return r > 256 && n <= 8192 ? 4 : 16; }

// Tuned source-split counts of the matrix-core kernel (yy_tune), 0 if none.
int tune_lookup(yy_ctx ctx, int32_t rp, int64_t n_pad, int32_t S, int32_t prec);
int64_t pair_mfma_npad(int64_t n);
int pair_mfma_rp(int32_t r, int32_t prec);

// Learned restart box (yy_proposal.hip): prepare writes the box chosen by the
// coverage and log-density checks and the decision words dec[0..2]; finish
// applies the prior-ESS check to the nodes generated from that box, switches
// the box back to the plain one when it fails (dec[1] = 1: regenerate), and
// writes `used`.
yy_status proposal_restart_prepare(yy_ctx ctx, yy_proposal p, int64_t n, int32_t r, const double* x_cur,
                                   const int64_t* idx, const double* mean, double R, double cover_min,
                                   double* box_lo, double* box_hi, int** dec_out);
yy_status proposal_restart_finish(yy_ctx ctx, yy_proposal p, int64_t n, int32_t r, const double* lw_new,
                                  const double* mean, double R, double ess_min, double* box_lo,
                                  double* box_hi, int* dec, int32_t* used);


// ---------------------------------------------------------------------------
// Argument sets of the batched kernels: the single-run kernels' parameters plus
// a predicate; one set per run, in device memory, for one launch over all runs.
struct loglik_args {
  int64_t n;
  int32_t r;
  int32_t m;
  int32_t obs;
  const double* H;
  double h_shift;
  const double* x;
  const double* dy;         // with kstep: the increments of all steps, dy_k = dy + (k - 1) m
  double dt;
  double rho2;
  double* logw;
  const int* pred;   // run only when *pred != 0 (NULL: always)
  const int32_t* kstep;     // device step counter k, or NULL
};

struct norm_max_args {
  int64_t n;
  const double* lw;
  double* pmax;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct norm_sumexp_args {
  int64_t n;
  int nb;
  const double* pmax;
  const double* lw;
  double* psum;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct norm_logz_args {
  int nb;
  const double* pmax;
  const double* psum;
  double* sc;
  double* logZ_step;
  double* logZ_acc;
  uint32_t* flags;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct norm_weights_args {
  int64_t n;
  int32_t r;
  int64_t rows;
  const double* sc;
  const double* x;
  double* lw;
  double* w;
  double* pw2;
  double* pmean;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct norm_final_args {
  int nb;
  int32_t r;
  const double* sc;
  const double* pw2;
  const double* pmean;
  double* mean;
  double* ess;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct rs_local_args {
  int64_t n;
  const double* w;
  unsigned long long* C;
  unsigned long long* tot;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct rs_offsets_args {
  int nb;
  unsigned long long* tot;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct rs_add_args {
  int64_t n;
  const unsigned long long* tot;
  unsigned long long* C;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct rs_search_args {
  int64_t n;
  int nb;
  const unsigned long long* tot;
  const unsigned long long* C;
  uint64_t U;
  int64_t* idx;
  uint32_t* flags;
  const int* pred;   // run only when *pred != 0 (NULL: always)
  const int32_t* kstep;     // with a device step counter: U = SplitMix64(key, k) >> 32
  uint64_t key;
};

struct box_plain_args {
  int32_t r;
  double R;
  const double* mean;
  double* box_lo;
  double* box_hi;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct restart_nodes_args {
  int64_t n;
  int32_t r;
  const uint32_t* codes;
  const double* mean;
  const double* box_lo;
  const double* box_hi;
  const int* only_if;
  double* x_new;
  double* logw_new;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct ess_check_args {
  const double* ess;
  double ess_min;
  uint32_t* flags;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct prepare_args {
  int64_t n;
  int64_t n_pad;
  int32_t r;
  int32_t rp;
  int32_t drift;
  const double* A;
  const double* x;
  const double* lo;
  const double* hi;
  float* xc32;
  float* f32;
  uint16_t* bf;
  float* f32t;
  double* node;
  int* bnd;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct prepare_scalars_args {
  int64_t n;
  int32_t r;
  int32_t nparts;    // per-block maxima written by the preparation (its block count)
  const double* lo;
  const double* hi;
  const double* node;
  double* scal;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct lw_max_args {
  int64_t n;
  const double* lw;
  const int* bnd;
  double* part;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

struct lw_convert_args {
  int64_t n;
  int nparts;
  const double* part;
  const double* lw;
  const int* bnd;
  float* lw2;
  double* ref_out;
  const int* pred;   // run only when *pred != 0 (NULL: always)
  long long* heavy;  // the heaviest source's index, or NULL
};

// Lower bounds of the pairwise rows' maxima (k_row_ref, yy_propagate.hip).
struct RowRefArgs {
  int64_t n;
  int32_t r, S, drift;
  const double* A;
  const double* x;
  const double* fw;       // whitened f rows [n][r], or null (then f from the drift)
  const float* lw2;
  const double* node;     // |f_i|^2 at node[n + i]
  const int* bnd;
  const long long* heavy; // [nheavy] the conversion blocks' candidates for j*
  int nheavy;
  long long* jstar;       // j*, the first valid source of maximal weight (-1: none)
  double* fstar;          // [r] f(x_j*)
  double kapd[YY_MAX_SCALES], taud[YY_MAX_SCALES];
  float* rref;            // [S][n] the rows' lower bounds
  float* rhv;             // [S][n] the exact term of the pair (i, j*) where the row counts it apart, else -inf
};

// j*, the first valid source of maximal weight, from the conversion blocks'
// candidates (one block), and f(x_j*) over the r coordinates.
__device__ __forceinline__ void k_heavy_body(const RowRefArgs& a) {
  __shared__ long long sj;
  if (threadIdx.x == 0) sj = LLONG_MAX;
  __syncthreads();
  long long m = LLONG_MAX;
  for (int p = threadIdx.x; p < a.nheavy; p += kBlock) m = a.heavy[p] < m ? a.heavy[p] : m;
  if (m != LLONG_MAX) atomicMin(&sj, m);
  __syncthreads();
  const long long js = sj == LLONG_MAX ? -1 : sj;
  if (threadIdx.x == 0) *a.jstar = js;
  if (js < 0) return;
  const double* xj = a.x + (size_t)js * a.r;
  for (int32_t k = threadIdx.x; k < a.r; k += kBlock) {
    double fk = 0.0;
    if (a.fw) {
      fk = a.fw[(size_t)js * a.r + k];
    } else if (a.drift == YY_F_COS) {
      fk = cos(xj[k]);
    } else if (a.drift == YY_F_PAPER_SINMIX) {
      const double xv = xj[k], xn = k + 1 < a.r ? xj[k + 1] : 0.0;
      fk = sin(xv) * (-0.5 * xv + 0.1 * xn) + sin(2.0 * xv) * (-0.3 * xv + 0.3 * xn);
    } else if (a.drift == YY_F_LINEAR) {
      double acc = 0.0;
      for (int32_t l = 0; l < a.r; ++l) acc = fma(a.A[(size_t)k * a.r + l], xj[l], acc);
      fk = acc;
    }
    a.fstar[k] = fk;
  }
}

// The source biases (k_src_bias) and, in one more block, j* with f(x_j*)
// (k_heavy_body): one launch, as neither reads what the other writes.
yy_status launch_src_bias_heavy(hipStream_t st, const PairArgs& a, const MfmaExtra& ex, const RowRefArgs& ra);

struct combine_args {
  CombineArgs a;
  const int* pred;   // run only when *pred != 0 (NULL: always)
};

yy_status launch_batched(hipStream_t st, const loglik_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const norm_max_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const norm_sumexp_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const norm_logz_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const norm_weights_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const norm_final_args* A, const int* pre, int nr, int total);
int norm_final_blocks(int32_t r);   // blocks of one k_norm_final launch
yy_status launch_batched(hipStream_t st, const rs_local_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const rs_offsets_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const rs_add_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const rs_search_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const box_plain_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const restart_nodes_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const ess_check_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const prepare_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const prepare_scalars_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const lw_max_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const lw_convert_args* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const RowRefArgs* A, const int* pre, int nr, int total);
yy_status launch_batched(hipStream_t st, const combine_args* A, const int* pre, int nr, int total);
// Source biases of many sets (the batched pairwise kernel's argument array).
yy_status launch_src_bias_batch(hipStream_t st, const void* sets, const int* pre, int nr, int total);

}  // namespace yy
