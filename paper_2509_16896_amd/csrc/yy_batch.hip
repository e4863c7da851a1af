// yy_batch.hip -- many independent filter runs stepped together, the step
// loop replayed through a HIP graph, and the autotuner of the pairwise
// kernel's source splits.
//
// Every kernel of a batch step is ONE launch over all runs: the block range of
// a launch is cut into one sub-range per run (the single-run call's grid), and
// each block runs the single-run kernel's body on its run's arguments, so the
// per-run arithmetic is exactly that of the single-run calls.  The pairwise
// kernel takes work items (run, target block, source split) in decreasing
// cost order.  Step counters and restart flags live on the device: restart
// kernels return at once in runs that do not restart at this step, so two
// consecutive steps form a graph that is captured once and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "yy_common.h"
#include "yy_internal.h"

namespace yy {

int tune_lookup(yy_ctx ctx, int32_t rp, int64_t n_pad, int32_t S, int32_t prec) {
  for (const auto& e : ctx->tune)
    if (e.rp == rp && e.n_pad == n_pad && e.S == S && e.prec == prec) return e.nsplit;
  return 0;
}

static void tune_store(yy_ctx ctx, int32_t rp, int64_t n_pad, int32_t S, int32_t prec, int32_t nsplit) {
  for (auto& e : ctx->tune)
    if (e.rp == rp && e.n_pad == n_pad && e.S == S && e.prec == prec) {
      e.nsplit = nsplit;
      return;
    }
  ctx->tune.push_back({rp, n_pad, S, prec, nsplit});
}

static bool is_mfma_prec(int32_t p) {
  return p == YY_PREC_BF16X3 || p == YY_PREC_BF16X3G || p == YY_PREC_BF16X3S || p == YY_PREC_BF16X3P ||
         p == YY_PREC_BF16X1 || p == YY_PREC_FP32_MFMA;
}

static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

struct BRun {
  yy_ctx rc = nullptr;
  yy_batch_run d{};
  DevBuf codes, x, lo, hi, lw[2], w, mean, ess, logZ_step, logZ_acc, logZ_scratch, hist, logZ_hist, ess_hist, idx,
      zero_r;
  int32_t k = 0;   // host mirror of the device step counter
  PropPlan plan;
};

// One batched launch: an argument set per run and the running block counts.
template <class T>
struct BLaunch {
  DevBuf args, pre;
  int nsets = 0, total = 0;
};

// Per-run control words on the device: step counter k and restart flag.
struct BCtl {
  int32_t k;
  int32_t restart;
  int32_t every;
  int32_t K;
};

__global__ void __launch_bounds__(kBlock) k_batch_advance(int nr, BCtl* __restrict__ c) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nr) return;
  const int32_t k = c[q].k + 1;
  c[q].k = k;
  c[q].restart = c[q].every > 0 && k % c[q].every == 0 && k < c[q].K;
}

struct record_args {
  int32_t r;
  const BCtl* ctl;
  const double* mean;
  const double* logZ_step;
  const double* ess;
  double* hist;
  double* logZ_hist;
  double* ess_hist;
};

// hist[k - 1] = mean, logZ_hist[k - 1] = logZ_k, ess_hist[k - 1] = ESS.
__global__ void __launch_bounds__(kBlock) k_batch_record(const record_args* __restrict__ A,
                                                         const int* __restrict__ pre, int nr) {
  const int q = batch_find(pre, nr, blockIdx.x);
  const record_args& a = A[q];
  const int32_t k = a.ctl->k;
  const int d = (blockIdx.x - pre[q]) * kBlock + threadIdx.x;
  if (d < a.r) a.hist[(size_t)(k - 1) * a.r + d] = a.mean[d];
  if (d == 0) {
    a.logZ_hist[k - 1] = *a.logZ_step;
    a.ess_hist[k - 1] = *a.ess;
  }
}

static int nblk(int64_t count) { return (int)((count + kBlock - 1) / kBlock); }

}  // namespace yy

struct yy_batch_s {
  yy_ctx ctx = nullptr;
  int32_t S = 0, prec = 0, max_split = 16, K = 0;
  double s[YY_MAX_SCALES] = {0, 0, 0, 0, 0, 0};
  double c[YY_MAX_SCALES + 1] = {0, 0, 0, 0, 0, 0, 0};
  bool have_c = false;
  std::vector<yy::BRun> runs;
  yy::DevBuf ctl;                  // BCtl [nruns]
  unsigned char* pinned = nullptr; // staging for uploads
  size_t pinned_bytes = 0;
  bool built = false;
  // each run's form of the pairwise sum: the batch's matrix-core form (the default), the plain FP32
  // form on the vector ALUs, or in a BF16X3P batch BF16X3G (BF16X3P with no screen and every tile
  // flagged) -- by yy_batch_tune with forms, or yy_batch_set_run_form
  std::vector<int32_t> form;
  // the pairwise launches: matrix-core runs, then vector-ALU runs by staging width (2, 4, 8, 16)
  yy::DevBuf d_sets, d_items;
  int nitems = 0;
  // BF16X3P: the screen's work lists (symmetric items for runs of more than kSymMinBlocks target
  // blocks, one-sided items for the others; group bounds and rechecks of the symmetric runs)
  yy::DevBuf d_scr_items, d_bound_items, d_recheck_items;
  yy::BatchScreen scr;
  // BF16X3P: per run a device int[2], [0] raised by the run's screen when it flags a tile in the step
  yy::DevBuf d_words;
  bool k64 = true;                 // every matrix-core run's K padding is a multiple of 64
  yy::DevBuf v_sets, v_items[4];
  int v_nitems[4] = {0, 0, 0, 0};
  yy::BLaunch<int> src_bias;       // argument sets = d_sets
  // parity-dependent launches (index k % 2 of the step)
  yy::BLaunch<yy::lw_max_args> lw_max[2];
  yy::BLaunch<yy::lw_convert_args> lw_convert[2];
  yy::BLaunch<yy::combine_args> combine[2];
  yy::BLaunch<yy::loglik_args> loglik[2];
  yy::BLaunch<yy::norm_max_args> nmax[2][2];        // [after restart][parity]
  yy::BLaunch<yy::norm_sumexp_args> nsum[2][2];
  yy::BLaunch<yy::norm_logz_args> nlogz[2][2];
  yy::BLaunch<yy::norm_weights_args> nwts[2][2];
  yy::BLaunch<yy::norm_final_args> nfin[2][2];
  yy::BLaunch<yy::restart_nodes_args> nodes[2];
  yy::BLaunch<yy::record_args> record;
  yy::BLaunch<yy::rs_local_args> rs_local;
  yy::BLaunch<yy::rs_offsets_args> rs_offsets;
  yy::BLaunch<yy::rs_add_args> rs_add;
  yy::BLaunch<yy::rs_search_args> rs_search;
  yy::BLaunch<yy::box_plain_args> box;
  yy::BLaunch<yy::prepare_args> prep;
  yy::BLaunch<yy::prepare_scalars_args> prep_scal;
  yy::BLaunch<yy::RowRefArgs> rowref;
  // graph of two consecutive steps, starting with parity g_parity
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_parity = -1;
};

namespace yy {

static yy_scales batch_scales(const yy_batch b) {
  yy_scales sc{};
  sc.S = b->S;
  sc.s = b->s;
  sc.c = b->have_c ? b->c : nullptr;
  return sc;
}

static yy_status staging(yy_batch b, size_t bytes) {
  if (bytes <= b->pinned_bytes) return YY_OK;
  if (b->pinned) (void)hipHostFree(b->pinned);
  b->pinned = nullptr;
  b->pinned_bytes = 0;
  YY_HIP(hipHostMalloc((void**)&b->pinned, bytes));
  b->pinned_bytes = bytes;
  return YY_OK;
}

// Synchronous upload through pinned staging (set-up time only).
static yy_status upload(yy_batch b, DevBuf& dst, const void* src, size_t bytes) {
  yy_status st = dst.ensure(bytes);
  if (st != YY_OK) return st;
  if ((st = staging(b, bytes)) != YY_OK) return st;
  YY_HIP(hipStreamSynchronize(b->ctx->stream));
  std::memcpy(b->pinned, src, bytes);
  YY_HIP(hipMemcpyAsync(dst.ptr, b->pinned, bytes, hipMemcpyHostToDevice, b->ctx->stream));
  YY_HIP(hipStreamSynchronize(b->ctx->stream));
  return YY_OK;
}

template <class T>
static yy_status build_launch(yy_batch b, BLaunch<T>& L, const std::vector<T>& A, const std::vector<int>& blocks) {
  std::vector<int> pre(blocks.size() + 1, 0);
  for (size_t q = 0; q < blocks.size(); ++q) pre[q + 1] = pre[q] + blocks[q];
  yy_status st;
  if (!A.empty() && (st = upload(b, L.args, A.data(), A.size() * sizeof(T))) != YY_OK) return st;
  if ((st = upload(b, L.pre, pre.data(), pre.size() * sizeof(int))) != YY_OK) return st;
  L.nsets = (int)blocks.size();
  L.total = pre.back();
  return YY_OK;
}

template <class T>
static yy_status run_launch(yy_batch b, const BLaunch<T>& L) {
  return launch_batched(b->ctx->stream, L.args.template as<T>(), L.pre.template as<int>(), L.nsets, L.total);
}

// Step 0 of one run: codes, nodes in the initial box with the N(0, I) prior, normalised.
static yy_status run_init(yy_batch b, BRun& R) {
  const yy_batch_run& d = R.d;
  const int32_t r = d.model.r;
  yy_status st;
  if ((st = yy_nodes_sobol(R.rc, r, d.n, 0, 1, d.seed, nullptr, nullptr, R.codes.as<uint32_t>(), nullptr)) != YY_OK)
    return st;
  YY_HIP(hipMemsetAsync(R.zero_r.ptr, 0, (size_t)r * sizeof(double), b->ctx->stream));
  YY_HIP(hipMemsetAsync(R.logZ_acc.ptr, 0, sizeof(double), b->ctx->stream));
  YY_HIP(hipMemsetAsync(R.logZ_scratch.ptr, 0, sizeof(double), b->ctx->stream));
  yy_restart_params rp{};
  rp.R = d.box_half;
  rp.seed = d.seed;
  if ((st = yy_restart(R.rc, d.n, r, R.codes.as<uint32_t>(), nullptr, nullptr, R.zero_r.as<double>(), nullptr, 0,
                       &rp, nullptr, R.lo.as<double>(), R.hi.as<double>(), R.x.as<double>(), R.lw[0].as<double>(),
                       nullptr)) != YY_OK)
    return st;
  R.k = 0;
  return yy_normalise_moments(R.rc, d.n, r, R.x.as<double>(), R.lw[0].as<double>(), R.w.as<double>(),
                              R.logZ_step.as<double>(), R.logZ_scratch.as<double>(), R.mean.as<double>(), nullptr,
                              R.ess.as<double>());
}

static yy_status reset_ctl(yy_batch b) {
  std::vector<BCtl> c(b->runs.size());
  for (size_t q = 0; q < b->runs.size(); ++q) c[q] = {0, 0, b->runs[q].d.restart_every, b->runs[q].d.K};
  return upload(b, b->ctl, c.data(), c.size() * sizeof(BCtl));
}

// A run of a BF16X3P batch set to BF16X3G takes BF16X3P's plan (row floor,
// pair with the heaviest source, flagged split pass) with no screen and every
// tile flagged: the split form on every tile, summed in BF16X3P's order.
static bool run_dense(yy_batch b, int q) {
  return b->prec == YY_PREC_BF16X3P && b->form[q] == YY_PREC_BF16X3G;
}
static int32_t run_plan_form(yy_batch b, int q) { return run_dense(b, q) ? b->prec : b->form[q]; }

// All launch descriptions: per-run plans (same split rule and scratch as the
// single-run calls), kernel argument sets for both step parities, work items.
static yy_status build(yy_batch b) {
  const yy_scales sc = batch_scales(b);
  const int nr = (int)b->runs.size();
  yy_status st;
  for (BRun& R : b->runs) {
    // a fixed node version: the prepared data is kept current by the batched
    // preparation after every restart, never by this call
    const int64_t jtl = (R.d.n + 127) / 128;
    const int split = (int)std::max<int64_t>(1, std::min<int64_t>(b->max_split, jtl));
    const int32_t form = run_plan_form(b, (int)(&R - b->runs.data()));
    if ((st = propagate_begin(R.rc, &R.d.model, &sc, form, R.d.n, R.x.as<double>(), 1, R.lo.as<double>(),
                              R.hi.as<double>(), R.d.dt, R.lw[0].as<double>(), R.lw[1].as<double>(), split,
                              R.plan)) != YY_OK)
      return st;
    // scratch of the steps that propagate_begin does not size
    const int nbn = norm_blocks(R.d.n);
    if ((st = R.rc->red2.ensure(((size_t)nbn * (3 + (size_t)R.d.model.r) + 4) * sizeof(double))) != YY_OK) return st;
    if ((st = R.rc->scan.ensure(((size_t)R.d.n + nblk(R.d.n) + 1) * sizeof(unsigned long long))) != YY_OK) return st;
  }
  // pairwise kernel argument sets and cost-ordered work items
  const size_t asz = pair_mfma_args_bytes();
  if ((st = b->d_words.ensure((size_t)2 * nr * sizeof(int))) != YY_OK) return st;
  YY_HIP(hipMemsetAsync(b->d_words.ptr, 0, (size_t)2 * nr * sizeof(int), b->ctx->stream));
  int* words = b->d_words.as<int>();
  std::vector<unsigned char> sets(nr * asz);
  struct Item {
    int run, tb, split;
    int64_t cost;
  };
  std::vector<Item> items;
  struct ScrItem {
    int4 it;
    int64_t cost;
  };
  std::vector<ScrItem> sitems;
  std::vector<int4> bitems, ritems;
  std::vector<int> bias_blocks(nr, 0);
  std::vector<ValuSet> vsets;
  std::vector<int4> vitems[4];
  for (int q = 0; q < nr; ++q) {
    const PropPlan& P = b->runs[q].plan;
    if (!P.mfma) {
      // the vector-ALU form: the single-run launch's blocks (64 targets, its source splits)
      ValuSet v{};
      v.a = P.a;
      v.per = valu_per(P.a);
      for (int s = 0; s < b->S; ++s) {
        v.taud[s] = P.taud[s];
        v.kapd[s] = P.kapd[s];
      }
      const int kc = valu_kc(P.a.r), cls = kc == 2 ? 0 : kc == 4 ? 1 : kc == 8 ? 2 : 3;
      const int64_t tiles = (P.n + 63) / 64;
      for (int sp = 0; sp < P.a.nsplit; ++sp)
        for (int64_t t = 0; t < tiles; ++t) vitems[cls].push_back(make_int4((int)vsets.size(), (int)t, sp, 0));
      vsets.push_back(v);
      continue;
    }
    MfmaExtra ex = P.ex;
    const bool dense = run_dense(b, q);
    if (b->prec == YY_PREC_BF16X3P && !dense) ex.flag_word = words + 2 * q;
    pair_mfma_fill_args(P.a, b->prec, ex, sets.data() + q * asz);
    bias_blocks[q] = nblk(P.ex.n_pad);
    const int64_t n = P.n, tbs = P.ex.n_pad / 256, jps = P.ex.j_per_split;
    // (in the partial-distance screened form a run whose screen spans 32 coordinates (r_p = 32) has a
    // weak screen that flags many of its tiles, so its split-pass items are costed as flagged and start
    // first instead of forming the launch's tail)
    const int64_t weak = b->prec == YY_PREC_BF16X3P && (P.a.rp <= 32 || dense) ? 64 : 1;
    for (int sp = 0; sp < P.a.nsplit; ++sp) {
      const int64_t j0 = (int64_t)sp * jps, j1 = std::min<int64_t>(j0 + jps, n);
      const int64_t cost = ((j1 - j0 + 127) / 128) * (int64_t)P.a.rp * weak;
      for (int64_t tb = 0; tb < tbs; ++tb) items.push_back({q, (int)tb, sp, cost});
    }
    if (dense) {
      // the split form on every tile: no screen; every flag set once here (no kernel writes them)
      YY_HIP(hipMemsetAsync(P.ex.flags, 1, (size_t)tbs * ((n + 127) / 128) * 8, b->ctx->stream));
    } else if (b->prec == YY_PREC_BF16X3P) {
      // the screen's items, costed in 128-source tiles (a symmetric tile carries both orientations'
      // verdicts: about 1.4 one-sided tiles)
      const int64_t jtl = (n + 127) / 128;
      if (P.ex.sym_items && P.ex.sym_nitems > 0 && P.ex.rref) {
        for (const int4& u : sym_work_items(tbs)) {
          const int64_t tiles = std::min<int64_t>(2 * (int64_t)u.z, jtl) - 2 * (int64_t)u.y;
          sitems.push_back({make_int4(q, u.x, u.y, u.z), tiles * 14 / 10});
        }
        const int64_t gblocks = (P.ex.n_pad / 64 + kBlock / 64 - 1) / (kBlock / 64);
        for (int64_t g = 0; g < gblocks; ++g) bitems.push_back(make_int4(q, (int)g, 0, 0));
        const int nb = 256;   // blocks striding over the run's list of doubted units (4 waves each;
                              // blocks past the list's end return at once)
        for (int g = 0; g < nb; ++g) ritems.push_back(make_int4(q, g, nb, 0));
      } else {
        for (int sp = 0; sp < P.a.nsplit; ++sp) {
          const int64_t j0 = (int64_t)sp * jps, j1 = std::min<int64_t>(j0 + jps, n);
          for (int64_t tb = 0; tb < tbs; ++tb)
            sitems.push_back({make_int4(q, (int)tb, sp, -1), (j1 - j0 + 127) / 128});
        }
      }
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  if (items.size() > (size_t)INT32_MAX) return fail(YY_ERR_UNSUPPORTED, "yy_batch: too many work items");
  std::vector<int4> it4(items.size());
  for (size_t t = 0; t < items.size(); ++t)
    it4[t] = make_int4(items[t].run, items[t].tb, items[t].split, (int)std::min<int64_t>(items[t].cost, INT32_MAX));
  if ((st = upload(b, b->d_sets, sets.data(), sets.size())) != YY_OK) return st;
  if ((st = upload(b, b->d_items, it4.data(), it4.size() * sizeof(int4))) != YY_OK) return st;
  b->nitems = (int)items.size();
  b->scr = yy::BatchScreen{};
  if (!sitems.empty()) {
    std::stable_sort(sitems.begin(), sitems.end(), [](const ScrItem& x, const ScrItem& y) { return x.cost > y.cost; });
    if (sitems.size() > (size_t)INT32_MAX) return fail(YY_ERR_UNSUPPORTED, "yy_batch: too many work items");
    std::vector<int4> s4(sitems.size());
    for (size_t t = 0; t < sitems.size(); ++t) s4[t] = sitems[t].it;
    if ((st = upload(b, b->d_scr_items, s4.data(), s4.size() * sizeof(int4))) != YY_OK) return st;
    b->scr.screen_items = b->d_scr_items.as<int4>();
    b->scr.nscreen = (int)s4.size();
  }
  if (!bitems.empty()) {
    if ((st = upload(b, b->d_bound_items, bitems.data(), bitems.size() * sizeof(int4))) != YY_OK) return st;
    b->scr.bound_items = b->d_bound_items.as<int4>();
    b->scr.nbound = (int)bitems.size();
    if ((st = upload(b, b->d_recheck_items, ritems.data(), ritems.size() * sizeof(int4))) != YY_OK) return st;
    b->scr.recheck_items = b->d_recheck_items.as<int4>();
    b->scr.nrecheck = (int)ritems.size();
  }
  b->k64 = true;
  for (const BRun& R : b->runs) b->k64 = b->k64 && (!R.plan.mfma || R.plan.a.rp % 64 == 0);
  if (!vsets.empty() && (st = upload(b, b->v_sets, vsets.data(), vsets.size() * sizeof(ValuSet))) != YY_OK) return st;
  for (int c = 0; c < 4; ++c) {
    b->v_nitems[c] = (int)vitems[c].size();
    if (!vitems[c].empty() && (st = upload(b, b->v_items[c], vitems[c].data(), vitems[c].size() * sizeof(int4))) != YY_OK)
      return st;
  }
  if ((st = build_launch(b, b->src_bias, std::vector<int>{}, bias_blocks)) != YY_OK) return st;

  const BCtl* ctl = b->ctl.as<BCtl>();
  for (int par = 0; par < 2; ++par) {
    // step k with k % 2 == par reads lw[(k + 1) % 2] and writes lw[k % 2]
    const int in = (par + 1) % 2, out = par;
    std::vector<lw_max_args> A1;
    std::vector<lw_convert_args> A2;
    std::vector<combine_args> A3;
    std::vector<loglik_args> A4;
    std::vector<norm_max_args> N1[2];
    std::vector<norm_sumexp_args> N2[2];
    std::vector<norm_logz_args> N3[2];
    std::vector<norm_weights_args> N4[2];
    std::vector<norm_final_args> N5[2];
    std::vector<restart_nodes_args> A5;
    std::vector<int> b_parts, b_n, b_ll, b_nb, b_one, b_r, b_nodes;
    for (int q = 0; q < nr; ++q) {
      BRun& R = b->runs[q];
      const yy_batch_run& d = R.d;
      const int64_t n = d.n;
      const int32_t r = d.model.r;
      const int* rflag = &ctl[q].restart;
      const Prepared& P = R.rc->prep;
      const int nparts = (int)std::min<int64_t>(nblk(n), 1024);
      double* d_part = R.rc->red.as<double>();
      double* d_lref = d_part + nparts;
      const double* lwi = R.lw[in].as<double>();
      double* lwo = R.lw[out].as<double>();
      A1.push_back({n, lwi, P.bnd.as<int>(), d_part, nullptr});
      A2.push_back({n, nparts, d_part, lwi, P.bnd.as<int>(), R.rc->lw2.as<float>(), d_lref, nullptr,
                    reinterpret_cast<long long*>(d_part + nparts + 8)});
      CombineArgs cb = R.plan.cb;
      cb.logw_in = lwi;
      cb.logw_out = lwo;
      // the run's flag word: with no tile flagged in the step the split pass wrote nothing and the
      // combination forms each target's self-pair split state itself (a run in the vector-ALU form, or
      // one with the split form on every tile, has none and combines every split)
      if (b->prec == YY_PREC_BF16X3P && R.plan.mfma && !run_dense(b, q)) cb.defer = b->d_words.as<int>() + 2 * q;
      A3.push_back({cb, nullptr});
      A4.push_back({n, r, d.model.m, d.model.obs, d.model.H, d.model.h_shift, R.x.as<double>(), d.dys, d.dt,
                    d.model.rho2, lwo, nullptr, &ctl[q].k});
      b_parts.push_back(nparts);
      b_n.push_back(nblk(n));
      int64_t blocks = (n + 3) / 4;
      if (blocks > 16384) blocks = 16384;
      b_ll.push_back((int)blocks);
      int64_t nb_nodes = blocks;
      if (nb_nodes * kBlock < r) nb_nodes = nblk(r);
      b_nodes.push_back((int)nb_nodes);
      const int nb = norm_blocks(n);
      const int64_t rows = (n + nb - 1) / nb;
      double* pmax = R.rc->red2.as<double>();
      double* psum = pmax + nb;
      double* pw2 = psum + nb;
      double* pmean = pw2 + nb;
      double* scv = pmean + (size_t)nb * r;
      for (int post = 0; post < 2; ++post) {
        const int* pr = post ? rflag : nullptr;
        double* acc = post ? R.logZ_scratch.as<double>() : R.logZ_acc.as<double>();
        N1[post].push_back({n, lwo, pmax, pr});
        N2[post].push_back({n, nb, pmax, lwo, psum, pr});
        N3[post].push_back({nb, pmax, psum, scv, R.logZ_step.as<double>(), acc, R.rc->d_flags, pr});
        // the restart prior's normalisation (post = 1) forms no moments and keeps no weights, as the
        // single-run filter's: x is not read
        N4[post].push_back({n, r, rows, scv, post ? nullptr : R.x.as<double>(), lwo, post ? nullptr : R.w.as<double>(),
                            pw2, pmean, pr});
        N5[post].push_back({nb, r, scv, pw2, pmean, post ? nullptr : R.mean.as<double>(), R.ess.as<double>(), pr});
      }
      b_nb.push_back(nb);
      b_one.push_back(1);
      b_r.push_back(norm_final_blocks(r));
      A5.push_back({n, r, R.codes.as<uint32_t>(), R.mean.as<double>(), R.lo.as<double>(), R.hi.as<double>(), nullptr,
                    R.x.as<double>(), lwo, rflag});
    }
    if ((st = build_launch(b, b->lw_max[par], A1, b_parts)) != YY_OK) return st;
    if ((st = build_launch(b, b->lw_convert[par], A2, b_parts)) != YY_OK) return st;
    if ((st = build_launch(b, b->combine[par], A3, b_n)) != YY_OK) return st;
    if ((st = build_launch(b, b->loglik[par], A4, b_ll)) != YY_OK) return st;
    for (int post = 0; post < 2; ++post) {
      if ((st = build_launch(b, b->nmax[post][par], N1[post], b_nb)) != YY_OK) return st;
      if ((st = build_launch(b, b->nsum[post][par], N2[post], b_nb)) != YY_OK) return st;
      if ((st = build_launch(b, b->nlogz[post][par], N3[post], b_one)) != YY_OK) return st;
      if ((st = build_launch(b, b->nwts[post][par], N4[post], b_nb)) != YY_OK) return st;
      if ((st = build_launch(b, b->nfin[post][par], N5[post], b_r)) != YY_OK) return st;
    }
    if ((st = build_launch(b, b->nodes[par], A5, b_nodes)) != YY_OK) return st;
  }
  // parity-independent launches
  std::vector<record_args> Rc;
  std::vector<rs_local_args> S1;
  std::vector<rs_offsets_args> S2;
  std::vector<rs_add_args> S3;
  std::vector<rs_search_args> S4;
  std::vector<box_plain_args> Bx;
  std::vector<prepare_args> Pp;
  std::vector<prepare_scalars_args> Ps;
  std::vector<RowRefArgs> Rr;
  std::vector<int> b_r, b_rs, b_one, b_prep, b_rr;
  for (int q = 0; q < nr; ++q) {
    BRun& R = b->runs[q];
    const yy_batch_run& d = R.d;
    const int64_t n = d.n;
    const int32_t r = d.model.r;
    const int* rflag = &ctl[q].restart;
    Prepared& P = R.rc->prep;
    Rc.push_back({r, &ctl[q], R.mean.as<double>(), R.logZ_step.as<double>(), R.ess.as<double>(), R.hist.as<double>(),
                  R.logZ_hist.as<double>(), R.ess_hist.as<double>()});
    const int nbr = nblk(n);
    unsigned long long* C = R.rc->scan.as<unsigned long long>();
    unsigned long long* tot = C + n;
    S1.push_back({n, R.w.as<double>(), C, tot, rflag});
    S2.push_back({nbr, tot, rflag});
    S3.push_back({n, tot, C, rflag});
    uint64_t key;
    {  // SplitMix64(seed, 2): the resampling stream of the run (as in yy_restart)
      uint64_t z = d.seed + 3ULL * 0x9E3779B97F4A7C15ULL;
      z ^= z >> 30;
      z *= 0xBF58476D1CE4E5B9ULL;
      z ^= z >> 27;
      z *= 0x94D049BB133111EBULL;
      key = z ^ (z >> 31);
    }
    S4.push_back({n, nbr, tot, C, 0, R.idx.as<int64_t>(), R.rc->d_flags, rflag, &ctl[q].k, key});
    Bx.push_back({r, d.R, R.mean.as<double>(), R.lo.as<double>(), R.hi.as<double>(), rflag});
    const bool bf = P.have_bf16, f32t = P.have_f32t;
    Pp.push_back({n, P.n_pad, r, P.rp, d.model.drift, d.model.A, R.x.as<double>(), R.lo.as<double>(),
                  R.hi.as<double>(), P.xc32.as<float>(), P.f32.as<float>(), bf ? P.bf.as<uint16_t>() : nullptr,
                  f32t ? P.f32t.as<float>() : nullptr, P.node.as<double>(), P.bnd.as<int>(), rflag});
    Ps.push_back({n, r, prepare_blocks(P.n_pad), R.lo.as<double>(), R.hi.as<double>(), P.node.as<double>(),
                  P.scal.as<double>(), rflag});
    b_r.push_back(nblk(r));
    b_rs.push_back(nbr);
    b_one.push_back(1);
    b_prep.push_back(prepare_blocks(P.n_pad));
    // the rows' lower bounds from this step's weights (as yy_propagate computes them)
    RowRefArgs ra{};
    ra.n = n;
    ra.r = r;
    ra.S = b->S;
    ra.drift = d.model.drift;
    ra.A = d.model.A;
    ra.x = R.x.as<double>();
    ra.fw = nullptr;
    ra.lw2 = R.rc->lw2.as<float>();
    ra.node = P.node.as<double>();
    ra.bnd = P.bnd.as<int>();
    const int nparts = (int)std::min<int64_t>(nblk(n), 1024);
    double* rbase = R.rc->red.as<double>();
    ra.heavy = reinterpret_cast<const long long*>(rbase + nparts + 8);
    ra.nheavy = nparts;
    ra.jstar = reinterpret_cast<long long*>(rbase + nparts + 1);
    if ((st = R.rc->fstar.ensure((size_t)r * sizeof(double))) != YY_OK) return st;
    ra.fstar = R.rc->fstar.as<double>();
    for (int s2 = 0; s2 < b->S; ++s2) {
      ra.kapd[s2] = R.plan.kapd[s2];
      ra.taud[s2] = R.plan.taud[s2];
    }
    // (the vector-ALU form has no row floor: no heavy source, no blocks)
    ra.rref = R.plan.mfma ? R.rc->rref.as<float>() : nullptr;
    ra.rhv = R.plan.mfma ? ra.rref + (size_t)b->S * n : nullptr;
    Rr.push_back(ra);
    b_rr.push_back(R.plan.mfma ? (int)((n + row_ref_targets(r, n) - 1) / row_ref_targets(r, n)) : 0);
  }
  if ((st = build_launch(b, b->record, Rc, b_r)) != YY_OK) return st;
  if ((st = build_launch(b, b->rs_local, S1, b_rs)) != YY_OK) return st;
  if ((st = build_launch(b, b->rs_offsets, S2, b_one)) != YY_OK) return st;
  if ((st = build_launch(b, b->rs_add, S3, b_rs)) != YY_OK) return st;
  if ((st = build_launch(b, b->rs_search, S4, b_rs)) != YY_OK) return st;
  if ((st = build_launch(b, b->box, Bx, b_r)) != YY_OK) return st;
  if ((st = build_launch(b, b->prep, Pp, b_prep)) != YY_OK) return st;
  if ((st = build_launch(b, b->prep_scal, Ps, b_one)) != YY_OK) return st;
  if ((st = build_launch(b, b->rowref, Rr, b_rr)) != YY_OK) return st;
  b->built = true;
  return YY_OK;
}

yy_status launch_batched(hipStream_t st, const record_args* A, const int* pre, int nr, int total) {
  if (total <= 0) return YY_OK;
  k_batch_record<<<total, kBlock, 0, st>>>(A, pre, nr);
  YY_LAUNCH_CHECK("k_batch_record");
  return YY_OK;
}

// The pairwise launches of a step: the matrix-core runs' work items, then the vector-ALU runs' per
// staging width.
static yy_status launch_pairwise(yy_batch b) {
  hipStream_t strm = b->ctx->stream;
  yy_status st;
  if (b->nitems > 0 &&
      (st = launch_pair_mfma_batch(strm, b->S, b->prec, b->d_sets.ptr, b->d_items.as<int4>(), b->nitems, b->k64,
                                   &b->scr)) !=
          YY_OK)
    return st;
  static const int kcs[4] = {2, 4, 8, 16};
  for (int c = 0; c < 4; ++c)
    if (b->v_nitems[c] > 0 &&
        (st = launch_pair_valu_batch(strm, b->S, kcs[c], b->v_sets.as<ValuSet>(), b->v_items[c].as<int4>(),
                                     b->v_nitems[c])) != YY_OK)
      return st;
  return YY_OK;
}

// One step of every run: 2 + 5 + 1 + 6 + 5 launches, plus 9 restart launches
// that return at once in runs not restarting this step.
static yy_status batch_step_impl(yy_batch b) {
  const int par = (b->runs[0].k + 1) % 2;
  hipStream_t strm = b->ctx->stream;
  const int nr = (int)b->runs.size();
  yy_status st;
  k_batch_advance<<<nblk(nr), kBlock, 0, strm>>>(nr, b->ctl.as<BCtl>());
  YY_LAUNCH_CHECK("k_batch_advance");
  if ((st = run_launch(b, b->lw_max[par])) != YY_OK) return st;
  if ((st = run_launch(b, b->lw_convert[par])) != YY_OK) return st;
  if ((st = launch_src_bias_batch(strm, b->d_sets.ptr, b->src_bias.pre.as<int>(), b->src_bias.nsets,
                                  b->src_bias.total)) != YY_OK)
    return st;
  if ((st = run_launch(b, b->rowref)) != YY_OK) return st;
  if ((st = timing_begin(b->ctx)) != YY_OK) return st;
  if ((st = launch_pairwise(b)) != YY_OK) return st;
  if ((st = timing_end(b->ctx)) != YY_OK) return st;
  if ((st = run_launch(b, b->combine[par])) != YY_OK) return st;
  if ((st = run_launch(b, b->loglik[par])) != YY_OK) return st;
  for (int post = 0; post < 2; ++post) {
    if (post == 1) {   // the restart of the runs whose flag is set, then their prior's normalisation
      if ((st = run_launch(b, b->rs_local)) != YY_OK) return st;
      if ((st = run_launch(b, b->rs_offsets)) != YY_OK) return st;
      if ((st = run_launch(b, b->rs_add)) != YY_OK) return st;
      if ((st = run_launch(b, b->rs_search)) != YY_OK) return st;
      if ((st = run_launch(b, b->box)) != YY_OK) return st;
      if ((st = run_launch(b, b->nodes[par])) != YY_OK) return st;
      if ((st = run_launch(b, b->prep)) != YY_OK) return st;
      if ((st = run_launch(b, b->prep_scal)) != YY_OK) return st;
    }
    if ((st = run_launch(b, b->nmax[post][par])) != YY_OK) return st;
    if ((st = run_launch(b, b->nsum[post][par])) != YY_OK) return st;
    if ((st = run_launch(b, b->nlogz[post][par])) != YY_OK) return st;
    if ((st = run_launch(b, b->nwts[post][par])) != YY_OK) return st;
    if ((st = run_launch(b, b->nfin[post][par])) != YY_OK) return st;
    if (post == 0 && (st = run_launch(b, b->record)) != YY_OK) return st;
  }
  for (BRun& R : b->runs) R.k += 1;
  return YY_OK;
}

static void drop_graph(yy_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->g_parity = -1;
}

static void release_launches(yy_batch b) {
  auto rel = [](auto& L) {
    L.args.release();
    L.pre.release();
  };
  rel(b->src_bias);
  for (int p = 0; p < 2; ++p) {
    rel(b->lw_max[p]);
    rel(b->lw_convert[p]);
    rel(b->combine[p]);
    rel(b->loglik[p]);
    rel(b->nodes[p]);
    for (int q = 0; q < 2; ++q) {
      rel(b->nmax[q][p]);
      rel(b->nsum[q][p]);
      rel(b->nlogz[q][p]);
      rel(b->nwts[q][p]);
      rel(b->nfin[q][p]);
    }
  }
  rel(b->record);
  rel(b->rs_local);
  rel(b->rs_offsets);
  rel(b->rs_add);
  rel(b->rs_search);
  rel(b->box);
  rel(b->prep);
  rel(b->prep_scal);
  rel(b->rowref);
}

}  // namespace yy

using namespace yy;

extern "C" yy_status yy_tune(yy_ctx ctx, int32_t count, const int32_t* r, const int64_t* n, const yy_scales* scales,
                             int32_t prec, int32_t reps, int32_t* nsplit_out) {
  if (!ctx || !r || !n || !scales) return fail(YY_ERR_ARG, "yy_tune: NULL argument");
  if (count < 0 || reps < 1 || reps > 1000) return fail(YY_ERR_ARG, "yy_tune: bad count or reps");
  if (!is_mfma_prec(prec)) return fail(YY_ERR_ARG, "yy_tune: prec must be a matrix-core form");
  if (scales->S < 1 || scales->S > 4) return fail(YY_ERR_ARG, "yy_tune: 1 to 4 scales");
  YY_HIP(hipSetDevice(ctx->device));
  if (capturing(ctx->stream)) return fail(YY_ERR_UNSUPPORTED, "yy_tune: stream is capturing");
  hipEvent_t e0, e1;
  YY_HIP(hipEventCreate(&e0));
  YY_HIP(hipEventCreate(&e1));
  yy_status st = YY_OK;
  for (int32_t t = 0; t < count && st == YY_OK; ++t) {
    if (r[t] < 1 || r[t] > YY_MAX_R || n[t] < 256 || n[t] > ((int64_t)1 << 24)) {
      st = fail(YY_ERR_ARG, "yy_tune: shape out of range");
      break;
    }
    DevBuf codes, x, lo, hi, lw0, lw1;
    const size_t nr = (size_t)n[t] * r[t];
    if ((st = codes.ensure(nr * 4)) != YY_OK || (st = x.ensure(nr * 8)) != YY_OK ||
        (st = lo.ensure((size_t)r[t] * 8)) != YY_OK || (st = hi.ensure((size_t)r[t] * 8)) != YY_OK ||
        (st = lw0.ensure((size_t)n[t] * 8)) != YY_OK || (st = lw1.ensure((size_t)n[t] * 8)) != YY_OK)
      break;
    std::vector<double> hlo(r[t], -1.0), hhi(r[t], 1.0);
    if (hipMemcpy(lo.ptr, hlo.data(), hlo.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(hi.ptr, hhi.data(), hhi.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(lw0.ptr, 0, (size_t)n[t] * 8, ctx->stream) != hipSuccess) {
      st = fail(YY_ERR_HIP, "yy_tune: set-up copies failed");
      break;
    }
    if ((st = yy_nodes_sobol(ctx, r[t], n[t], 0, 1, 12345, lo.as<double>(), hi.as<double>(), codes.as<uint32_t>(),
                             x.as<double>())) != YY_OK)
      break;
    yy_model m{};
    m.r = r[t];
    m.m = r[t];
    m.drift = YY_F_COS;
    m.obs = YY_H_CUBE;
    m.q = 0.09;
    m.rho2 = 0.09;
    const int64_t jtl = (n[t] + 127) / 128;
    int best = 0;
    float best_ms = 0.f;
    for (int cand = 1; cand <= 256 && cand <= jtl && st == YY_OK; cand *= 2) {
      PropPlan plan;
      st = propagate_begin(ctx, &m, scales, prec, n[t], x.as<double>(), 777, lo.as<double>(), hi.as<double>(), 0.01,
                           lw0.as<double>(), lw1.as<double>(), cand, plan);
      if (st != YY_OK) break;
      if ((st = launch_pair_mfma(ctx->stream, plan.a, plan.prec, plan.ex)) != YY_OK) break;   // warm-up
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(YY_ERR_HIP, "yy_tune: event"); break; }
      for (int q = 0; q < reps && st == YY_OK; ++q) st = launch_pair_mfma(ctx->stream, plan.a, plan.prec, plan.ex);
      if (st != YY_OK) break;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = fail(YY_ERR_HIP, "yy_tune: event");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best == 0 || ms < best_ms) {
        best = plan.a.nsplit;
        best_ms = ms;
      }
    }
    if (st == YY_OK) {
      tune_store(ctx, pair_mfma_rp(r[t], prec), pair_mfma_npad(n[t]), scales->S, prec, best);
      if (nsplit_out) nsplit_out[t] = best;
    }
    (void)hipStreamSynchronize(ctx->stream);
    codes.release();
    x.release();
    lo.release();
    hi.release();
    lw0.release();
    lw1.release();
  }
  ctx->prep.valid = false;   // the synthetic node sets are gone
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

extern "C" yy_status yy_batch_create(yy_ctx ctx, int32_t nruns, const yy_batch_run* runs, const yy_scales* scales,
                                     int32_t prec, int32_t max_split, yy_batch* out) {
  if (!ctx || !runs || !scales || !out) return fail(YY_ERR_ARG, "yy_batch_create: NULL argument");
  *out = nullptr;
  if (nruns < 1 || nruns > 4096) return fail(YY_ERR_ARG, "yy_batch_create: nruns out of range");
  if (!is_mfma_prec(prec)) return fail(YY_ERR_ARG, "yy_batch_create: prec must be a matrix-core form");
  if (scales->S < 1 || scales->S > 4 || !scales->s) return fail(YY_ERR_ARG, "yy_batch_create: 1 to 4 scales");
  if (scales->form != YY_FORM_PUSH) return fail(YY_ERR_UNSUPPORTED, "yy_batch_create: the batched step is push-form only");
  if (max_split < 0 || max_split > 256) return fail(YY_ERR_ARG, "yy_batch_create: max_split out of range");
  for (int32_t q = 0; q < nruns; ++q) {
    const yy_batch_run& d = runs[q];
    yy_status st = validate_model(&d.model);
    if (st != YY_OK) return st;
    if (d.model.noise) return fail(YY_ERR_UNSUPPORTED, "yy_batch_create: general noise coefficients are single-run only");
    if (d.n < 1 || d.n > ((int64_t)1 << 31)) return fail(YY_ERR_ARG, "yy_batch_create: n out of range");
    if (!(d.dt > 0.0) || !(d.box_half > 0.0) || !(d.R > 0.0)) return fail(YY_ERR_ARG, "yy_batch_create: dt, box, R");
    if (d.K < 1 || d.restart_every < 0 || !d.dys) return fail(YY_ERR_ARG, "yy_batch_create: K, restart, dys");
    if (d.K != runs[0].K) return fail(YY_ERR_ARG, "yy_batch_create: all runs of a batch take the same K");
  }
  YY_HIP(hipSetDevice(ctx->device));
  yy_batch b = new yy_batch_s();
  b->ctx = ctx;
  b->S = scales->S;
  b->prec = prec;
  b->K = runs[0].K;
  b->max_split = max_split > 0 ? max_split : 16;
  for (int s = 0; s < b->S; ++s) b->s[s] = scales->s[s];
  if (scales->c) {
    b->have_c = true;
    for (int s = 0; s <= b->S; ++s) b->c[s] = scales->c[s];
  }
  b->runs.resize(nruns);
  b->form.resize(nruns);
  for (int32_t q = 0; q < nruns; ++q) b->form[q] = prec;
  yy_status st = YY_OK;
  for (int32_t q = 0; q < nruns && st == YY_OK; ++q) {
    BRun& R = b->runs[q];
    R.d = runs[q];
    const int64_t n = R.d.n;
    const int32_t r = R.d.model.r;
    if ((st = yy_create(&R.rc, ctx->device, ctx->stream)) != YY_OK) break;
    const size_t nr = (size_t)n * r;
    DevBuf* bufs[] = {&R.codes, &R.x, &R.lo, &R.hi, &R.lw[0], &R.lw[1], &R.w, &R.mean, &R.ess, &R.logZ_step,
                      &R.logZ_acc, &R.logZ_scratch, &R.hist, &R.logZ_hist, &R.ess_hist, &R.idx, &R.zero_r};
    const size_t sizes[] = {nr * 4, nr * 8, (size_t)r * 8, (size_t)r * 8, (size_t)n * 8, (size_t)n * 8,
                            (size_t)n * 8, (size_t)r * 8, 8, 8, 8, 8, (size_t)R.d.K * r * 8, (size_t)R.d.K * 8,
                            (size_t)R.d.K * 8, (size_t)n * 8, (size_t)r * 8};
    for (size_t t = 0; t < sizeof(sizes) / sizeof(sizes[0]) && st == YY_OK; ++t) st = bufs[t]->ensure(sizes[t]);
    if (st == YY_OK) st = run_init(b, R);
  }
  if (st == YY_OK) st = reset_ctl(b);
  if (st == YY_OK) st = build(b);   // also prepares the initial nodes
  if (st == YY_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(YY_ERR_HIP, "yy_batch_create");
  if (st != YY_OK) {
    yy_batch_destroy(b);
    return st;
  }
  *out = b;
  return YY_OK;
}

extern "C" yy_status yy_batch_destroy(yy_batch b) {
  if (!b) return YY_OK;
  if (b->ctx) {
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
  }
  drop_graph(b);
  release_launches(b);
  for (BRun& R : b->runs) {
    DevBuf* bufs[] = {&R.codes, &R.x, &R.lo, &R.hi, &R.lw[0], &R.lw[1], &R.w, &R.mean, &R.ess, &R.logZ_step,
                      &R.logZ_acc, &R.logZ_scratch, &R.hist, &R.logZ_hist, &R.ess_hist, &R.idx, &R.zero_r};
    for (DevBuf* p : bufs) p->release();
    if (R.rc) yy_destroy(R.rc);
    R.rc = nullptr;
  }
  b->ctl.release();
  b->d_sets.release();
  b->d_items.release();
  b->d_scr_items.release();
  b->d_words.release();
  b->d_bound_items.release();
  b->d_recheck_items.release();
  b->v_sets.release();
  for (int c = 0; c < 4; ++c) b->v_items[c].release();
  if (b->pinned) (void)hipHostFree(b->pinned);
  delete b;
  return YY_OK;
}

extern "C" yy_status yy_batch_reset(yy_batch b) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_reset: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  yy_status st;
  for (BRun& R : b->runs)
    if ((st = run_init(b, R)) != YY_OK) return st;
  if ((st = reset_ctl(b)) != YY_OK) return st;
  // build() prepares the initial nodes again
  for (BRun& R : b->runs) R.rc->prep.valid = false;
  return build(b);
}

extern "C" yy_status yy_batch_step(yy_batch b) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_step: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  if (b->runs[0].k >= b->K) return fail(YY_ERR_ARG, "yy_batch_step: every run has taken its K steps");
  return batch_step_impl(b);
}

extern "C" yy_status yy_batch_run_graph(yy_batch b, int32_t k_end) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_run_graph: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  const int32_t k0 = b->runs[0].k;
  if (k_end > b->K) return fail(YY_ERR_ARG, "yy_batch_run_graph: k_end beyond K");
  if (k_end <= k0) return YY_OK;
  if (b->ctx->timing) return fail(YY_ERR_UNSUPPORTED, "yy_batch_run_graph: disable timing first");
  hipStream_t st = b->ctx->stream;
  if (st == nullptr) return fail(YY_ERR_UNSUPPORTED, "yy_batch_run_graph: graph capture needs a created stream");
  const int pairs = (k_end - k0) / 2;
  if (pairs > 0) {
    const int parity = (k0 + 1) % 2;
    if (!b->exec || b->g_parity != parity) {
      drop_graph(b);
      YY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      // the captured steps advance the host-side step counters, but nothing runs until a replay: put
      // every counter back as it was, whether or not both steps were recorded
      std::vector<int32_t> k_saved(b->runs.size());
      for (size_t i = 0; i < b->runs.size(); ++i) k_saved[i] = b->runs[i].k;
      yy_status s = batch_step_impl(b);
      if (s == YY_OK) s = batch_step_impl(b);
      for (size_t i = 0; i < b->runs.size(); ++i) b->runs[i].k = k_saved[i];
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (s != YY_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != YY_OK ? s : hip_fail(ec, "hipStreamEndCapture");
      }
      b->graph = g;
      const hipError_t ei = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        b->exec = nullptr;
        drop_graph(b);
        return hip_fail(ei, "hipGraphInstantiate");
      }
      b->g_parity = parity;
    }
    for (int p = 0; p < pairs; ++p) YY_HIP(hipGraphLaunch(b->exec, st));
    for (BRun& R : b->runs) R.k += 2 * pairs;
  }
  if ((k_end - k0) % 2) return batch_step_impl(b);
  return YY_OK;
}

extern "C" yy_status yy_batch_tune(yy_batch b, int32_t reps, int32_t forms, int32_t* best_out) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_tune: NULL batch");
  if (reps < 1 || reps > 1000) return fail(YY_ERR_ARG, "yy_batch_tune: reps out of range");
  YY_HIP(hipSetDevice(b->ctx->device));
  hipStream_t st = b->ctx->stream;
  if (capturing(st)) return fail(YY_ERR_UNSUPPORTED, "yy_batch_tune: stream is capturing");
  drop_graph(b);
  hipEvent_t e0, e1;
  YY_HIP(hipEventCreate(&e0));
  YY_HIP(hipEventCreate(&e1));
  yy_status s = YY_OK;
  // (1) each run's form: its pairwise call (on its own context, as the batch plans it) timed in the
  // batch's matrix-core form and in the candidates `forms` names -- the plain FP32 form on the vector
  // ALUs (bit 0), the split form on every tile in a BF16X3P batch (bit 1, BF16X3G's single-run call
  // standing for it) -- the fastest is kept.  Runs of the same (r, n) share the first one's choice.
  if (forms & 3) {
    const yy_scales sc = batch_scales(b);
    std::vector<std::pair<std::pair<int32_t, int64_t>, int32_t>> chosen;
    for (size_t q = 0; q < b->runs.size() && s == YY_OK; ++q) {
      BRun& R = b->runs[q];
      if (!(forms & 1) && b->form[q] == YY_PREC_FP32) continue;   // keeps the vector-ALU form
      const std::pair<int32_t, int64_t> key(R.d.model.r, R.d.n);
      int32_t pick = -1;
      for (const auto& c : chosen)
        if (c.first == key) pick = c.second;
      if (pick < 0) {
        float ms_f[3] = {0.f, 0.f, 0.f};
        int32_t cand[3] = {b->prec, 0, 0};
        int nc = 1;
        if (forms & 1) cand[nc++] = YY_PREC_FP32;
        if ((forms & 2) && b->prec == YY_PREC_BF16X3P) cand[nc++] = YY_PREC_BF16X3G;
        for (int f = 0; f < nc && s == YY_OK; ++f) {
          const int64_t jtl = (R.d.n + 127) / 128;
          const int split = (int)std::max<int64_t>(1, std::min<int64_t>(b->max_split, jtl));
          PropPlan plan;
          s = propagate_begin(R.rc, &R.d.model, &sc, cand[f], R.d.n, R.x.as<double>(), 1, R.lo.as<double>(),
                              R.hi.as<double>(), R.d.dt, R.lw[0].as<double>(), R.lw[1].as<double>(), split, plan);
          if (s == YY_OK) s = propagate_pair(R.rc, plan);   // warm-up
          if (s == YY_OK && hipEventRecord(e0, st) != hipSuccess) s = fail(YY_ERR_HIP, "yy_batch_tune: event");
          for (int t = 0; t < reps && s == YY_OK; ++t) s = propagate_pair(R.rc, plan);
          if (s == YY_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            s = fail(YY_ERR_HIP, "yy_batch_tune: event");
          if (s == YY_OK) (void)hipEventElapsedTime(&ms_f[f], e0, e1);
        }
        if (s != YY_OK) break;
        int best_f = 0;
        for (int f = 1; f < nc; ++f)
          if (ms_f[f] < ms_f[best_f]) best_f = f;
        pick = cand[best_f];
        chosen.push_back({key, pick});
      }
      b->form[q] = pick;
    }
  }
  const int keep = b->max_split;
  int best = keep;
  float best_ms = -1.f;
  // (2) the matrix-core runs' source splits
  for (int cand = 1; cand <= 64 && s == YY_OK; cand *= 2) {
    b->max_split = cand;
    if ((s = build(b)) != YY_OK) break;
    if ((s = launch_pairwise(b)) != YY_OK) break;
    if (hipEventRecord(e0, st) != hipSuccess) { s = fail(YY_ERR_HIP, "yy_batch_tune: event"); break; }
    for (int q = 0; q < reps && s == YY_OK; ++q) s = launch_pairwise(b);
    if (s != YY_OK) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      s = fail(YY_ERR_HIP, "yy_batch_tune: event");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      best = cand;
    }
  }
  b->max_split = s == YY_OK ? best : keep;
  const yy_status s2 = build(b);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != YY_OK) return s;
  if (s2 != YY_OK) return s2;
  if (best_out) *best_out = best;
  return YY_OK;
}

extern "C" yy_status yy_batch_results(yy_batch b, int32_t run, double* mean_hist, double* logZ_hist,
                                      double* ess_hist) {
  if (!b || run < 0 || run >= (int32_t)b->runs.size()) return fail(YY_ERR_ARG, "yy_batch_results: bad run");
  YY_HIP(hipSetDevice(b->ctx->device));
  const BRun& R = b->runs[run];
  hipStream_t st = b->ctx->stream;
  const size_t K = (size_t)R.d.K, r = (size_t)R.d.model.r;
  if (mean_hist) YY_HIP(hipMemcpyAsync(mean_hist, R.hist.ptr, K * r * 8, hipMemcpyDeviceToDevice, st));
  if (logZ_hist) YY_HIP(hipMemcpyAsync(logZ_hist, R.logZ_hist.ptr, K * 8, hipMemcpyDeviceToDevice, st));
  if (ess_hist) YY_HIP(hipMemcpyAsync(ess_hist, R.ess_hist.ptr, K * 8, hipMemcpyDeviceToDevice, st));
  return YY_OK;
}

extern "C" yy_status yy_batch_run_form(yy_batch b, int32_t run, int32_t* prec) {
  if (!b || run < 0 || run >= (int32_t)b->runs.size() || !prec) return fail(YY_ERR_ARG, "yy_batch_run_form: bad run");
  *prec = b->form[run];
  return YY_OK;
}

extern "C" yy_status yy_batch_set_run_form(yy_batch b, int32_t run, int32_t prec) {
  if (!b || run < 0 || run >= (int32_t)b->runs.size()) return fail(YY_ERR_ARG, "yy_batch_set_run_form: bad run");
  if (prec != b->prec && prec != YY_PREC_FP32 && !(b->prec == YY_PREC_BF16X3P && prec == YY_PREC_BF16X3G))
    return fail(YY_ERR_ARG,
                "yy_batch_set_run_form: the batch's matrix-core form, YY_PREC_FP32, or in a BF16X3P batch "
                "YY_PREC_BF16X3G");
  YY_HIP(hipSetDevice(b->ctx->device));
  if (capturing(b->ctx->stream)) return fail(YY_ERR_UNSUPPORTED, "yy_batch_set_run_form: stream is capturing");
  if (b->form[run] == prec) return YY_OK;
  drop_graph(b);
  b->form[run] = prec;
  return build(b);
}

extern "C" yy_status yy_batch_screen_count(yy_batch b, int32_t run, int64_t* flagged, int64_t* tiles) {
  if (!b || run < 0 || run >= (int32_t)b->runs.size()) return fail(YY_ERR_ARG, "yy_batch_screen_count: bad run");
  return yy_screen_count(b->runs[run].rc, flagged, tiles);
}

extern "C" yy_status yy_batch_step_count(yy_batch b, int32_t* k) {
  if (!b || !k) return fail(YY_ERR_ARG, "yy_batch_step_count: NULL argument");
  *k = b->runs[0].k;
  return YY_OK;
}
