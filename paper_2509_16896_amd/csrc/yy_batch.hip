// yy_batch.hip -- many independent filter runs stepped together, the step
// loop replayed through a HIP graph, and the autotuner of the pairwise
// kernel's source splits.
//
// A batch step runs, per run, the preparation, source weights and biases of
// yy_propagate, then ONE matrix-core pairwise launch over the work items
// (run, target block, source split) of every run, sorted by decreasing cost,
// then per run the combination, the log-likelihood update, the normalisation
// and, every restart_every steps, the plain restart.  Each run has its own
// context (scratch, prepared nodes) on the batch's stream, so the per-run
// arithmetic is exactly that of the single-run calls.
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
  return p == YY_PREC_BF16X3 || p == YY_PREC_BF16X3G || p == YY_PREC_BF16X1 || p == YY_PREC_FP32_MFMA;
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
  int cur = 0;
  uint64_t version = 0;
  int32_t k = 0;
  PropPlan plan;
};

// Host-side state that the step code advances (restored around graph launches).
struct BRunState {
  int cur;
  uint64_t version;
  int32_t k;
  Prepared prep;
};

}  // namespace yy

struct yy_batch_s {
  yy_ctx ctx = nullptr;
  int32_t S = 0, prec = 0, max_split = 16;
  double s[YY_MAX_SCALES] = {0, 0, 0, 0, 0, 0};
  double c[YY_MAX_SCALES + 1] = {0, 0, 0, 0, 0, 0, 0};
  bool have_c = false;
  std::vector<yy::BRun> runs;
  // the batched launch: per-run kernel arguments and work items
  yy::DevBuf d_sets, d_items;
  std::vector<unsigned char> h_sets;
  std::vector<int> set_run;        // run of each set in the current launch
  unsigned char* pinned = nullptr; // staging for uploads
  size_t pinned_bytes = 0;
  int nitems = 0;
  // graph of steps k0+1 .. k1
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t g_k0 = -1, g_k1 = -1;
  std::vector<yy::BRunState> g_pre, g_post;
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
  R.cur = 0;
  if ((st = yy_restart(R.rc, d.n, r, R.codes.as<uint32_t>(), nullptr, nullptr, R.zero_r.as<double>(), nullptr, 0,
                       &rp, nullptr, R.lo.as<double>(), R.hi.as<double>(), R.x.as<double>(), R.lw[0].as<double>(),
                       nullptr)) != YY_OK)
    return st;
  R.version += 1;
  R.k = 0;
  return yy_normalise_moments(R.rc, d.n, r, R.x.as<double>(), R.lw[0].as<double>(), R.w.as<double>(),
                              R.logZ_step.as<double>(), R.logZ_scratch.as<double>(), R.mean.as<double>(), nullptr,
                              R.ess.as<double>());
}

// Per-run kernel arguments and the cost-ordered work items of the active runs;
// uploads them when they differ from the last upload.
static yy_status prepare_launch(yy_batch b, const std::vector<int>& active) {
  const size_t asz = pair_mfma_args_bytes();
  std::vector<unsigned char> sets(active.size() * asz);
  for (size_t t = 0; t < active.size(); ++t)
    pair_mfma_fill_args(b->runs[active[t]].plan.a, b->prec, b->runs[active[t]].plan.ex, sets.data() + t * asz);
  if (sets == b->h_sets && active == b->set_run) return YY_OK;
  if (capturing(b->ctx->stream))
    return fail(YY_ERR_UNSUPPORTED, "yy_batch: the batched launch changed while capturing a graph");
  struct Item {
    int run, tb, split;
    int64_t cost;
  };
  std::vector<Item> items;
  for (size_t t = 0; t < active.size(); ++t) {
    const PropPlan& P = b->runs[active[t]].plan;
    const int64_t n = P.n, tbs = P.ex.n_pad / 256, jps = P.ex.j_per_split;
    for (int sp = 0; sp < P.a.nsplit; ++sp) {
      const int64_t j0 = (int64_t)sp * jps, j1 = std::min<int64_t>(j0 + jps, n);
      const int64_t cost = ((j1 - j0 + 127) / 128) * (int64_t)P.a.rp;
      for (int64_t tb = 0; tb < tbs; ++tb) items.push_back({(int)t, (int)tb, sp, cost});
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  if (items.size() > (size_t)INT32_MAX) return fail(YY_ERR_UNSUPPORTED, "yy_batch: too many work items");
  yy_status st;
  if ((st = b->d_sets.ensure(sets.size())) != YY_OK) return st;
  if ((st = b->d_items.ensure(items.size() * sizeof(int4))) != YY_OK) return st;
  if ((st = staging(b, sets.size() + items.size() * sizeof(int4))) != YY_OK) return st;
  // the previous upload may still be in flight from the staging buffer
  YY_HIP(hipStreamSynchronize(b->ctx->stream));
  std::memcpy(b->pinned, sets.data(), sets.size());
  int4* it4 = reinterpret_cast<int4*>(b->pinned + sets.size());
  for (size_t q = 0; q < items.size(); ++q)
    it4[q] = make_int4(items[q].run, items[q].tb, items[q].split, (int)std::min<int64_t>(items[q].cost, INT32_MAX));
  YY_HIP(hipMemcpyAsync(b->d_sets.ptr, b->pinned, sets.size(), hipMemcpyHostToDevice, b->ctx->stream));
  YY_HIP(hipMemcpyAsync(b->d_items.ptr, it4, items.size() * sizeof(int4), hipMemcpyHostToDevice, b->ctx->stream));
  YY_HIP(hipStreamSynchronize(b->ctx->stream));
  b->h_sets.swap(sets);
  b->set_run = active;
  b->nitems = (int)items.size();
  return YY_OK;
}

static int run_split(const yy_batch b, const BRun& R) {
  const int64_t jtl = (R.d.n + 127) / 128;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b->max_split, jtl));
}

// Phase 1 for the active runs (those below their K).
static yy_status begin_all(yy_batch b, std::vector<int>& active) {
  const yy_scales sc = batch_scales(b);
  active.clear();
  for (int q = 0; q < (int)b->runs.size(); ++q) {
    BRun& R = b->runs[q];
    if (R.k >= R.d.K) continue;
    yy_status st = propagate_begin(R.rc, &R.d.model, &sc, b->prec, R.d.n, R.x.as<double>(), R.version,
                                   R.lo.as<double>(), R.hi.as<double>(), R.d.dt, R.lw[R.cur].as<double>(),
                                   R.lw[1 - R.cur].as<double>(), run_split(b, R), R.plan);
    if (st != YY_OK) return st;
    active.push_back(q);
  }
  return YY_OK;
}

static yy_status batch_step_impl(yy_batch b) {
  std::vector<int> active;
  yy_status st = begin_all(b, active);
  if (st != YY_OK || active.empty()) return st;
  if ((st = prepare_launch(b, active)) != YY_OK) return st;
  if ((st = timing_begin(b->ctx)) != YY_OK) return st;
  if ((st = launch_pair_mfma_batch(b->ctx->stream, b->S, b->prec, b->d_sets.ptr, b->d_items.as<int4>(), b->nitems)) !=
      YY_OK)
    return st;
  if ((st = timing_end(b->ctx)) != YY_OK) return st;
  hipStream_t strm = b->ctx->stream;
  for (int q : active) {
    BRun& R = b->runs[q];
    const yy_batch_run& d = R.d;
    const int32_t r = d.model.r;
    if ((st = propagate_end(R.rc, R.plan)) != YY_OK) return st;
    R.cur = 1 - R.cur;
    const int32_t k = R.k + 1;
    double* lw = R.lw[R.cur].as<double>();
    if ((st = yy_loglik_update(R.rc, &d.model, d.n, R.x.as<double>(), d.dys + (size_t)(k - 1) * d.model.m, d.dt,
                               lw)) != YY_OK)
      return st;
    if ((st = yy_normalise_moments(R.rc, d.n, r, R.x.as<double>(), lw, R.w.as<double>(), R.logZ_step.as<double>(),
                                   R.logZ_acc.as<double>(), R.mean.as<double>(), nullptr, R.ess.as<double>())) != YY_OK)
      return st;
    YY_HIP(hipMemcpyAsync(R.hist.as<double>() + (size_t)(k - 1) * r, R.mean.ptr, (size_t)r * sizeof(double),
                          hipMemcpyDeviceToDevice, strm));
    YY_HIP(hipMemcpyAsync(R.logZ_hist.as<double>() + (k - 1), R.logZ_step.ptr, sizeof(double),
                          hipMemcpyDeviceToDevice, strm));
    YY_HIP(hipMemcpyAsync(R.ess_hist.as<double>() + (k - 1), R.ess.ptr, sizeof(double), hipMemcpyDeviceToDevice,
                          strm));
    R.k = k;
    if (d.restart_every > 0 && k % d.restart_every == 0 && k < d.K) {
      yy_restart_params rp{};
      rp.R = d.R;
      rp.seed = d.seed;
      if ((st = yy_restart(R.rc, d.n, r, R.codes.as<uint32_t>(), nullptr, R.w.as<double>(), R.mean.as<double>(),
                           R.ess.as<double>(), k, &rp, R.idx.as<int64_t>(), R.lo.as<double>(), R.hi.as<double>(),
                           R.x.as<double>(), lw, nullptr)) != YY_OK)
        return st;
      R.version += 1;
      if ((st = yy_normalise_moments(R.rc, d.n, r, R.x.as<double>(), lw, R.w.as<double>(), R.logZ_step.as<double>(),
                                     R.logZ_scratch.as<double>(), R.mean.as<double>(), nullptr,
                                     R.ess.as<double>())) != YY_OK)
        return st;
    }
  }
  return YY_OK;
}

static void drop_graph(yy_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->g_k0 = b->g_k1 = -1;
  b->g_pre.clear();
  b->g_post.clear();
}

static std::vector<BRunState> snapshot(const yy_batch b) {
  std::vector<BRunState> v;
  for (const BRun& R : b->runs) v.push_back({R.cur, R.version, R.k, R.rc->prep});
  return v;
}

static void restore(yy_batch b, const std::vector<BRunState>& v) {
  for (size_t q = 0; q < v.size(); ++q) {
    BRun& R = b->runs[q];
    R.cur = v[q].cur;
    R.version = v[q].version;
    R.k = v[q].k;
    R.rc->prep = v[q].prep;
  }
}

static bool same_state(const yy_batch b, const std::vector<BRunState>& v) {
  if (v.size() != b->runs.size()) return false;
  for (size_t q = 0; q < v.size(); ++q) {
    const BRun& R = b->runs[q];
    if (R.cur != v[q].cur || R.version != v[q].version || R.k != v[q].k) return false;
  }
  return true;
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
      tune_store(ctx, pair_mfma_rp(r[t]), pair_mfma_npad(n[t]), scales->S, prec, best);
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
  if (max_split < 0 || max_split > 256) return fail(YY_ERR_ARG, "yy_batch_create: max_split out of range");
  for (int32_t q = 0; q < nruns; ++q) {
    const yy_batch_run& d = runs[q];
    yy_status st = validate_model(&d.model);
    if (st != YY_OK) return st;
    if (d.n < 1 || d.n > ((int64_t)1 << 31)) return fail(YY_ERR_ARG, "yy_batch_create: n out of range");
    if (!(d.dt > 0.0) || !(d.box_half > 0.0) || !(d.R > 0.0)) return fail(YY_ERR_ARG, "yy_batch_create: dt, box, R");
    if (d.K < 1 || d.restart_every < 0 || !d.dys) return fail(YY_ERR_ARG, "yy_batch_create: K, restart, dys");
  }
  YY_HIP(hipSetDevice(ctx->device));
  yy_batch b = new yy_batch_s();
  b->ctx = ctx;
  b->S = scales->S;
  b->prec = prec;
  b->max_split = max_split > 0 ? max_split : 16;
  for (int s = 0; s < b->S; ++s) b->s[s] = scales->s[s];
  if (scales->c) {
    b->have_c = true;
    for (int s = 0; s <= b->S; ++s) b->c[s] = scales->c[s];
  }
  b->runs.resize(nruns);
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
  for (BRun& R : b->runs) {
    DevBuf* bufs[] = {&R.codes, &R.x, &R.lo, &R.hi, &R.lw[0], &R.lw[1], &R.w, &R.mean, &R.ess, &R.logZ_step,
                      &R.logZ_acc, &R.logZ_scratch, &R.hist, &R.logZ_hist, &R.ess_hist, &R.idx, &R.zero_r};
    for (DevBuf* p : bufs) p->release();
    if (R.rc) yy_destroy(R.rc);
    R.rc = nullptr;
  }
  b->d_sets.release();
  b->d_items.release();
  if (b->pinned) (void)hipHostFree(b->pinned);
  delete b;
  return YY_OK;
}

extern "C" yy_status yy_batch_reset(yy_batch b) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_reset: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  for (BRun& R : b->runs) {
    yy_status st = run_init(b, R);
    if (st != YY_OK) return st;
  }
  return YY_OK;
}

extern "C" yy_status yy_batch_step(yy_batch b) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_step: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  return batch_step_impl(b);
}

extern "C" yy_status yy_batch_run_graph(yy_batch b, int32_t k_end) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_run_graph: NULL batch");
  YY_HIP(hipSetDevice(b->ctx->device));
  const int32_t k0 = b->runs[0].k;
  for (const BRun& R : b->runs) {
    if (R.k != k0) return fail(YY_ERR_ARG, "yy_batch_run_graph: runs are at different steps");
    if (k_end > R.d.K) return fail(YY_ERR_ARG, "yy_batch_run_graph: k_end beyond a run's K");
    if (R.d.restart_every > 0 && k0 < R.d.restart_every)
      return fail(YY_ERR_ARG, "yy_batch_run_graph: take restart_every eager steps first");
  }
  if (k0 < 1) return fail(YY_ERR_ARG, "yy_batch_run_graph: take eager steps first");
  if (k_end <= k0) return YY_OK;
  if (b->ctx->timing) return fail(YY_ERR_UNSUPPORTED, "yy_batch_run_graph: disable timing first");
  hipStream_t st = b->ctx->stream;
  if (st == nullptr) return fail(YY_ERR_UNSUPPORTED, "yy_batch_run_graph: graph capture needs a created stream");
  if (!(b->exec && b->g_k0 == k0 && b->g_k1 == k_end && same_state(b, b->g_pre))) {
    drop_graph(b);
    // any change of the batched launch must be uploaded before the capture
    std::vector<int> active;
    yy_status s0 = begin_all(b, active);
    if (s0 == YY_OK) s0 = prepare_launch(b, active);
    if (s0 != YY_OK) return s0;
    // the graph prepares its first step's nodes itself, so that it does not
    // depend on what was prepared before a launch
    for (BRun& R : b->runs) R.rc->prep.valid = false;
    b->g_pre = snapshot(b);
    YY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    yy_status s = YY_OK;
    for (int32_t k = k0 + 1; k <= k_end && s == YY_OK; ++k) s = batch_step_impl(b);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (s != YY_OK || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      restore(b, b->g_pre);
      b->g_pre.clear();
      return s != YY_OK ? s : hip_fail(ec, "hipStreamEndCapture");
    }
    b->graph = g;
    const hipError_t ei = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      b->exec = nullptr;
      restore(b, b->g_pre);
      drop_graph(b);
      return hip_fail(ei, "hipGraphInstantiate");
    }
    b->g_post = snapshot(b);
    b->g_k0 = k0;
    b->g_k1 = k_end;
    restore(b, b->g_pre);
  }
  YY_HIP(hipGraphLaunch(b->exec, st));
  restore(b, b->g_post);
  return YY_OK;
}

extern "C" yy_status yy_batch_tune(yy_batch b, int32_t reps, int32_t* best_out) {
  if (!b) return fail(YY_ERR_ARG, "yy_batch_tune: NULL batch");
  if (reps < 1 || reps > 1000) return fail(YY_ERR_ARG, "yy_batch_tune: reps out of range");
  YY_HIP(hipSetDevice(b->ctx->device));
  hipStream_t st = b->ctx->stream;
  if (capturing(st)) return fail(YY_ERR_UNSUPPORTED, "yy_batch_tune: stream is capturing");
  drop_graph(b);
  hipEvent_t e0, e1;
  YY_HIP(hipEventCreate(&e0));
  YY_HIP(hipEventCreate(&e1));
  const int keep = b->max_split;
  int best = keep;
  float best_ms = -1.f;
  yy_status s = YY_OK;
  for (int cand = 1; cand <= 64 && s == YY_OK; cand *= 2) {
    b->max_split = cand;
    std::vector<int> active;
    if ((s = begin_all(b, active)) != YY_OK || active.empty()) break;
    if ((s = prepare_launch(b, active)) != YY_OK) break;
    if ((s = launch_pair_mfma_batch(st, b->S, b->prec, b->d_sets.ptr, b->d_items.as<int4>(), b->nitems)) != YY_OK)
      break;
    if (hipEventRecord(e0, st) != hipSuccess) { s = fail(YY_ERR_HIP, "yy_batch_tune: event"); break; }
    for (int q = 0; q < reps && s == YY_OK; ++q)
      s = launch_pair_mfma_batch(st, b->S, b->prec, b->d_sets.ptr, b->d_items.as<int4>(), b->nitems);
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
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s == YY_OK && best_out) *best_out = best;
  return s;
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

extern "C" yy_status yy_batch_step_count(yy_batch b, int32_t* k) {
  if (!b || !k) return fail(YY_ERR_ARG, "yy_batch_step_count: NULL argument");
  int32_t m = 0;
  for (const BRun& R : b->runs) m = std::max(m, R.k);
  *k = m;
  return YY_OK;
}
