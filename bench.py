#!/usr/bin/env python3
"""Throughput of the improved Yau-Yau filter step on one MI355X.

A step is one pass of the whole hot path over the synthetic cubic-sensor
workload r=1000, n=65536 (f = cos, h = x^3, noise std 0.3, dt = 0.005, kernel
scales {1, 2, 4}, restart every 2 steps with R = 0.3): yy_propagate,
yy_loglik_update, yy_normalise_moments and, every second step, yy_restart with
its normalisation.  Inputs (nodes, weights, observation increments) are
resident in HBM before the timed region starts.

Prints one JSON line: steps/s; the propagation's matrix-core work per second
on the work it executes (in the screened forms: the screen's products for
every pair plus the method's products 2 n^2 r P on the tiles the screen
keeps, P = 2 products x.x and x.f for several scales); the roofline of the
pairwise kernel on that basis (timed with HIP events on the library's
stream) beside the method's own work 2 n^2 r P expressed as the time a dense
evaluation would take at the matrix-core peak; a second roofline record for
the split form on every tile (BF16X3G); the plain FP32 form timed beside it;
and the FP64 oracle on a bounded sample of the same step on the host cores.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "filter steps/sec + propagation TFLOP/s at r=1000,n=65536 vs plain FP32, same error"
PEAK_TFLOPS = {"bf16x3": 2500.0, "bf16x3g": 2500.0, "bf16x3s": 2500.0, "bf16x3p": 2500.0, "bf16x1": 2500.0,
               "fp32_mfma": 157.3}
VALU_FP32_PEAK = 78.6   # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 disabled
# matrix-core products executed per algorithmic product (x.x and x.f each count once)
EXEC_PER_ALG = {"bf16x3": 3.0, "bf16x3g": 2.0, "bf16x1": 1.0, "fp32_mfma": 1.0}
PRE_K = 64   # coordinates of the partial-distance screen (BF16X3P)
SYM_MIN_BLOCKS = 32   # one run in BF16X3P with more target blocks of 256 than this takes the symmetric screen
# (r, n) of the paper's large-scale test (the workloads module holds the same list)
PAPER_E1 = ((10, 100), (50, 300), (100, 500), (300, 800), (600, 1000), (1000, 2000))
PAIR_SRC = os.path.join(ROOT, "paper_2509_16896_amd", "csrc", "yy_pair_mfma.hip")
TRAFFIC_FILES = {
    "bf16x3p": os.path.join(ROOT, "profiles", "k_pair_mfma_cubic_r1000_n65536_traffic.md"),
    "bf16x3g": os.path.join(ROOT, "profiles", "k_pair_mfma_bf16x3g_cubic_r1000_n65536_traffic.md"),
}
DENSE_FORM = "bf16x3g"   # the split form on every tile: the second roofline record


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def alg_flops(w) -> float:
    """The method's pairwise products per propagation: 2 n^2 r per product, x.x and (S > 1) x.f."""
    P = 1 if len(w.scales) == 1 else 2
    return 2.0 * w.n * w.n * w.r * P


def screen_pairs(n, prec, r=1000):
    """Pairs whose screen product is formed: every ordered pair, or, where the symmetric screen
    runs (BF16X3P with more than SYM_MIN_BLOCKS target blocks of 256 and r > 32, whose screen spans
    64 coordinates), the 256 x 128 tiles of each target block A against the source tiles from 2A on
    (G = X X^T serves both orientations of a block pair; diagonal blocks are formed whole)."""
    tbs = -(-n // 256)
    if prec != "bf16x3p" or tbs <= SYM_MIN_BLOCKS or r <= 32:
        return float(n) * n
    jtl = -(-n // 128)
    return 256.0 * 128.0 * sum(jtl - 2 * a for a in range(tbs))


def screened_work(w, prec, flagged, tiles):
    """(algorithmic, executed) matrix-core flop of one propagation in a screened form: the
    screen's product x.x for every pair it forms (screen_pairs) over the coordinates it uses
    (all r for BF16X3S, the first 64 for BF16X3P; the x.f term is bounded, not formed), plus
    the method's products on the flagged tiles, which the split form executes twice over
    (three BF16 products for x.x, one for x.f)."""
    k = w.r if prec == "bf16x3s" else min(PRE_K, w.r)
    screen = 2.0 * screen_pairs(w.n, prec, w.r) * k
    split = alg_flops(w) * flagged / max(tiles, 1)
    return screen + split, screen + 2.0 * split


def run_gpu(w, dys, prec, warmup, steps, timing=True, proposal_params=None, form="push", operator=False):
    import torch
    from paper_2509_16896_amd import yy
    from paper_2509_16896_amd.filter import GpuFilter

    f = GpuFilter(w, prec=prec, proposal_params=proposal_params, form=form, operator=operator)
    f.set_observations(dys)
    f.init()
    k = 0
    for _ in range(warmup):
        k += 1
        f.step(k, restart=(w.restart_every and k % w.restart_every == 0))
    torch.cuda.synchronize()
    if timing:
        yy.yy_timing_enable(f.ctx, True)
        yy.yy_timing_read(f.ctx)
    t0 = time.perf_counter()
    for _ in range(steps):
        k += 1
        f.step(k, restart=(w.restart_every and k % w.restart_every == 0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches = yy.yy_timing_read(f.ctx) if timing else (0.0, 0)
    yy.yy_timing_enable(f.ctx, False)
    return f, k, t1 - t0, ms, launches


def kernel_source_hash() -> str:
    with open(PAIR_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def recorded_traffic(prec: str):
    """HBM bytes per launch of the pairwise kernel from the committed counter summary, or None
    when the summary is missing, covers another form, or the kernel source changed since."""
    path = TRAFFIC_FILES.get(prec)
    if path is None or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_") and "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("traffic_source_hash") != kernel_source_hash() or vals.get("traffic_prec") != prec:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def traffic_probe(w, prec):
    """Run under rocprofv3 --pmc: one device copy of exactly 1 GiB (the calibration kernel),
    then one yy_propagate of the workload (the pairwise kernel)."""
    import torch
    from paper_2509_16896_amd import yy
    from paper_2509_16896_amd.filter import GpuFilter

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    from paper_2509_16896_amd import workloads as W

    xs, dys = W.simulate(w)
    f = GpuFilter(w, prec=prec)
    f.set_observations(dys)
    f.init()
    out = torch.empty(w.n, dtype=torch.float64, device=f.dev)
    yy.yy_propagate(f.ctx, f.model, f.scales, prec, w.n, f.x, f.version, f.lo, f.hi, w.dt, f.lw[f.cur], out)
    torch.cuda.synchronize()
    f.close()
    log(f"[bench] traffic probe done ({prec}, source hash {kernel_source_hash()})")


def cpu_baseline(w, f, k_last, target_s=15.0, form="push"):
    """The oracle on a bounded sample of one step of the same workload: the propagation of a
    few target rows (extrapolated to all n rows) plus the full correction and normalisation."""
    import numpy as np
    import torch

    import oracle
    from oracle import filter as ofilter

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    torch.cuda.synchronize()
    x = f.x.cpu().numpy().reshape(w.n, w.r)
    lw = f.lw[f.cur].cpu().numpy()
    lo, hi = f.lo.cpu().numpy(), f.hi.cpu().numpy()
    model = ofilter.model_of(w)
    s = np.asarray(w.scales, float)
    c = oracle.kernel_coefficients(s)
    oform = oracle.FORM_PULL if form == "pull" else oracle.FORM_PUSH
    rng = np.random.default_rng(0)
    order = rng.permutation(w.n)
    # target rows in growing batches until about target_s seconds of oracle work are done
    done, batch, t_rows, parts = 0, 16, 0.0, []
    while t_rows < target_s and done < w.n:
        rows_b = np.sort(order[done:done + batch])
        t0 = time.perf_counter()
        ref_b, _ = oracle.propagate_rows_ex(model, s, c, x, lo, hi, w.dt, lw, rows_b, form=oform)
        t_rows += time.perf_counter() - t0
        parts.append((rows_b, ref_b))
        done += len(rows_b)
        batch *= 2
    rows = np.concatenate([p[0] for p in parts])
    ref_rows = np.concatenate([p[1] for p in parts])
    nrows = len(rows)
    dy = f.dys[k_last - 1].cpu().numpy()
    t0 = time.perf_counter()
    lw2 = oracle.loglik_update(model, x, dy, w.dt, lw)
    oracle.normalise_moments(x, lw2, 0.0, want_cov=False)
    t_rest = time.perf_counter() - t0
    t_step = t_rows * (w.n / nrows) + t_rest
    return dict(value=1.0 / t_step, unit="steps/s", cores=threads, kind="oracle", cpu_model=host_cpu_model(),
                logical_cpus=os.cpu_count(),
                sample=f"FP64 oracle: propagation of {nrows} of {w.n} target rows of one step "
                       f"({t_rows:.1f} s, extrapolated to all rows) + full correction/normalisation "
                       f"({t_rest:.2f} s)"), (rows, ref_rows, x, lw, lo, hi)


def sampled_parity(w, f, prec, sample):
    """GPU propagation of the same state compared with the oracle's rows."""
    import numpy as np
    import torch
    from scipy.special import logsumexp

    from paper_2509_16896_amd import yy

    rows, ref_rows, x, lw, lo, hi = sample
    out = torch.empty(w.n, dtype=torch.float64, device=f.dev)
    yy.yy_propagate(f.ctx, f.model, f.scales, prec, w.n, f.x, f.version, f.lo, f.hi, w.dt, f.lw[f.cur], out)
    got = out.cpu().numpy()
    fin = np.isfinite(ref_rows)
    # both sides are row samples of the same vector: compare relative to the full GPU normaliser
    z = logsumexp(got[np.isfinite(got)])
    rel = np.abs(got[rows][fin] - ref_rows[fin]) / np.maximum(1.0, np.abs(ref_rows[fin] - z))
    return float(np.max(rel)) if rel.size else float("nan")


# the paper's table of its large-scale test: (r, n) -> time for 1000 steps (s), RMSE, ME, each mean and
# standard deviation over 20 runs, on the paper's own hardware (context, not a target)
PAPER_E1_TABLE = {10: ((0.271, 0.023), (0.165, 0.002), (0.160, 0.002)),
                  50: ((1.006, 0.026), (0.368, 0.001), (0.365, 0.001)),
                  100: ((4.824, 0.095), (0.523, 0.005), (0.520, 0.005)),
                  300: ((16.833, 0.374), (0.964, 0.034), (0.955, 0.033)),
                  600: ((37.160, 0.065), (1.376, 0.049), (1.356, 0.046)),
                  1000: ((150.540, 6.431), (1.609, 0.013), (1.582, 0.012))}


def main_e1_table(args):
    """The paper's large-scale test at its six (r, n) sizes: 1000 filter steps per run, `seeds` runs
    per size (truth path, observations and node scramble keyed by the seed), the wall time of the
    1000 steps on the GPU (state initialised and observations resident before the clock starts), RMSE
    and ME to the true path; printed beside the paper's own table."""
    import numpy as np
    import torch

    from paper_2509_16896_amd import workloads as W
    from paper_2509_16896_amd.filter import GpuFilter

    out = []
    for r, n in PAPER_E1:
        times, rmses, mes = [], [], []
        for sd in range(args.seeds):
            w = W.paper_e1(r, seed=sd)
            xs, dys = W.simulate(w)
            f = GpuFilter(w, prec=args.prec_given or w.precision)
            try:
                f.set_observations(dys)
                f.init()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for k in range(1, w.K + 1):
                    f.step(k)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                est = f.hist.cpu().numpy()
            finally:
                f.close()
            rmses.append(W.rmse(est, xs[1:]))
            mes.append(W.mean_error(est, xs[1:]))
        pt, pr, pm = PAPER_E1_TABLE[r]
        row = {"r": r, "n": n, "steps": 1000, "runs": args.seeds, "precision": args.prec_given or w.precision,
               "time_s": [round(float(np.mean(times)), 4), round(float(np.std(times)), 4)],
               "rmse": [round(float(np.mean(rmses)), 4), round(float(np.std(rmses)), 4)],
               "me": [round(float(np.mean(mes)), 4), round(float(np.std(mes)), 4)],
               "paper_time_s": list(pt), "paper_rmse": list(pr), "paper_me": list(pm)}
        out.append(row)
        log(f"[bench] paper E1 r={r} n={n}: {row['time_s'][0]:.3f} s per 1000 steps, RMSE {row['rmse'][0]:.3f}, "
            f"ME {row['me'][0]:.3f} (paper: {pt[0]} s, {pr[0]}, {pm[0]})")
    print(json.dumps({"workload": "paper_e1_table", "data": "synthetic",
                      "sizes": out}), flush=True)


def main_form_compare(args):
    """Push form against the pull form of eq. kernel (divergence in closed form) on the cubic
    sensor r=2 (n=1024, fixed box), the linear-Gaussian r=10 (n=4096) and the cubic sensor r=100
    (n=16384): `seeds` full runs each, RMSE and ME to the true path and steps/s of the whole step.
    The plain FP32 form where r < 32 (the matrix cores need r >= 32), the split form BF16X3G
    otherwise (the screened forms are push-form only)."""
    import numpy as np
    import torch

    from paper_2509_16896_amd import workloads as W
    from paper_2509_16896_amd.filter import GpuFilter

    out = []
    for w0 in (W.cubic_r2(), W.linear_r10(), W.cubic_r100()):
        prec = "fp32" if w0.r < 32 else "bf16x3g"
        row = {"workload": w0.name, "r": w0.r, "n": w0.n, "K": w0.K, "precision": prec}
        for form in ("push", "pull"):
            rm, me, sps = [], [], []
            for sd in range(args.seeds):
                w = dataclasses.replace(w0, seed=sd)
                xs, dys = W.simulate(w)
                f = GpuFilter(w, prec=prec, form=form)
                try:
                    f.set_observations(dys)
                    f.init()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for k in range(1, w.K + 1):
                        f.step(k)
                    torch.cuda.synchronize()
                    sps.append(w.K / (time.perf_counter() - t0))
                    est = f.hist.cpu().numpy()
                finally:
                    f.close()
                rm.append(W.rmse(est, xs[1:]))
                me.append(W.mean_error(est, xs[1:]))
            row[form] = {"rmse": [round(float(np.mean(rm)), 4), round(float(np.std(rm)), 4)],
                         "me": [round(float(np.mean(me)), 4), round(float(np.std(me)), 4)],
                         "steps_per_s": round(float(np.mean(sps)), 1)}
            log(f"[bench] {w0.name} {form}: RMSE {row[form]['rmse'][0]:.4f}, ME {row[form]['me'][0]:.4f}, "
                f"{row[form]['steps_per_s']} steps/s")
        out.append(row)
    print(json.dumps({"workload": "push_vs_pull", "runs": args.seeds, "data": "synthetic", "rows": out}), flush=True)


def main_batch(args):
    """The batch of 64 uneven cubic-sensor runs: aggregate filter steps/s of the graph-replayed
    step loop, beside the same batch stepped eagerly and the runs filtered one after another."""
    import numpy as np
    import torch

    from paper_2509_16896_amd import workloads as W
    from paper_2509_16896_amd import yy
    from paper_2509_16896_amd.batch import Batch
    from paper_2509_16896_amd.filter import GpuFilter

    ws = W.batch_runs(64, seed=0)
    K = ws[0].K
    dys = [W.simulate(w)[1] for w in ws]
    alg = sum(2.0 * w.n * w.n * w.r * 2 for w in ws)   # per batched pairwise launch
    log(f"[bench] batch of {len(ws)} runs, r in [{min(w.r for w in ws)}, {max(w.r for w in ws)}], "
        f"n in [{min(w.n for w in ws)}, {max(w.n for w in ws)}], K={K}, prec={args.prec}")
    bt = Batch(ws, dys, prec=args.prec)
    t0 = time.perf_counter()
    if args.batch_forms == "rule":
        for q, w in enumerate(ws):
            if w.r < 32:
                bt.set_run_form(q, "fp32")
    for _ in range(4):     # a state past the first restarts: the screens' cost depends on the weights
        bt.step()
    # (in BF16X3P each run's screen is also timed against the split form on every tile)
    best = bt.tune(reps=2, forms=args.batch_forms == "tuned",
                   dense=args.prec == "bf16x3p" and args.batch_forms != "rule")
    tune_s = time.perf_counter() - t0
    forms = [bt.run_form(q) for q in range(len(ws))]
    mfma_runs = [q for q, fm in enumerate(forms) if fm != "fp32"]
    dense_runs = [q for q in mfma_runs if forms[q] != args.prec]
    log(f"[bench] tuned: {len(ws) - len(mfma_runs)} runs on the vector ALUs (plain FP32), {len(mfma_runs)} in "
        f"{args.prec} ({len(dense_runs)} of them with the split form on every tile, no screen: "
        f"{sorted((ws[q].r, ws[q].n) for q in dense_runs)}); max source splits per run {best} ({tune_s:.2f} s)")

    def run_eager():
        bt.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(K):
            bt.step()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def run_graph():
        bt.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        bt.step()
        bt.step()
        bt.run_graph(K)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    run_graph()                       # capture + instantiate + first launch
    t_graph = min(run_graph() for _ in range(max(1, args.steps // 10)))
    t_eager = run_eager()
    # the pairwise launch alone (HIP events on the batch's stream)
    bt.reset()
    bt.step()
    bt.step()
    yy.yy_timing_enable(bt.ctx, True)
    yy.yy_timing_read(bt.ctx)
    for _ in range(4):
        bt.step()
    ms, cnt = yy.yy_timing_read(bt.ctx)
    yy.yy_timing_enable(bt.ctx, False)
    kms = ms / max(cnt, 1)
    kernel = "k_pair_mfma_batch"
    dense = alg
    # the matrix-core roofline counts the matrix-core runs' work; the vector-ALU runs' launch is inside
    # the same timed region, so the rate is a lower bound
    alg = sum(2.0 * ws[q].n * ws[q].n * ws[q].r * 2 for q in mfma_runs)
    if args.prec in ("bf16x3s", "bf16x3p"):
        # each run's screen products plus the method's products on its flagged tiles
        # (a run with the split form on every tile forms no screen products)
        counts = {q: bt.screen_count(q) for q in mfma_runs}
        alg = sum(alg_flops(ws[q]) if q in dense_runs else screened_work(ws[q], args.prec, fl, tl)[0]
                  for q, (fl, tl) in counts.items())
        kernel = ("k_tgt_bound_batch, k_pair_prescreen_batch (symmetric items for runs of more than 32 target "
                  "blocks with r > 32, one-sided items for the others) and k_sym_recheck_batch"
                  if args.prec == "bf16x3p" else "k_pair_screen_batch") + \
            ", then k_pair_mfma_batch (split form) on flagged tiles"
        log(f"[bench] screens flagged {sum(c[0] for c in counts.values())} of "
            f"{sum(c[1] for c in counts.values())} tiles")
    if len(mfma_runs) < len(ws):
        kernel += "; k_pair_valu_batch for the runs on the vector ALUs"
    bt.close()
    # the same runs one after another through the single-run calls
    t_seq = 0.0
    for w, d, fm in zip(ws, dys, forms):
        f = GpuFilter(w, prec=fm)
        f.set_observations(d)
        f.init()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(1, K + 1):
            f.step(k)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t
        f.close()
    steps = len(ws) * K
    achieved = alg / (kms * 1e-3) / 1e12
    line = {
        "metric": "aggregate filter steps/s, batch of 64 uneven cubic-sensor runs", "value": round(steps / t_graph, 2),
        "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": 2, "ms_per_step": round(1e3 * t_graph / K, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "batch64_cubic_r10-200_n2048-32768", "runs": len(ws), "K": K,
                   "precision": args.prec, "max_split": best, "forms": args.batch_forms,
                   "runs_on_vector_alus": len(ws) - len(mfma_runs),
                   "runs_split_on_every_tile": len(dense_runs)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS[args.prec],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[args.prec], 4), "traffic": None,
                     "kernel": kernel, "kernel_ms": round(kms, 3),
                     "work_basis": ("each matrix-core run's screen products plus 2 n^2 r P on its flagged tiles "
                                    "(on every tile for a run with no screen)"
                                    if args.prec in ("bf16x3s", "bf16x3p") else "2 n^2 r P of every matrix-core run")
                     + "; the timed launches include the vector-ALU runs",
                     "method_dense_at_peak_ms": round(dense / (PEAK_TFLOPS[args.prec] * 1e12) * 1e3, 4)},
        "eager_steps_per_s": round(steps / t_eager, 2),
        "sequential_single_run_steps_per_s": round(steps / t_seq, 2),
        "tune_s": round(tune_s, 2),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default=None,
                    choices=["fp32", "fp32_mfma", "bf16x3", "bf16x3g", "bf16x3s", "bf16x3p", "bf16x1"],
                    help="form of the pairwise sum (default: bf16x3p)")
    ap.add_argument("--other-forms", default="bf16x3s,bf16x3g,bf16x3,bf16x1",
                    help="matrix-core forms whose pairwise kernel is also timed ('none' to skip)")
    ap.add_argument("--baseline-prec", default="fp32_mfma", help="plain FP32 form timed beside ('none' to skip)")
    ap.add_argument("--baseline-steps", type=int, default=4)
    ap.add_argument("--workload", default="cubic_r1000",
                    choices=["cubic_r1000", "cubic_r100", "batch64"] + [f"paper_e1_r{r}" for r, _ in PAPER_E1])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--proposal", default="none", choices=["learned", "none"],
                    help="restart box: the plain box (default) or the learned MLP proposal, trained before timing; "
                         "on held-out runs of the cubic r=100 n=16384 and r=1000 n=4096 filters its checks never "
                         "passed, so the default step does not pay for it")
    ap.add_argument("--train-runs", type=int, default=2, help="plain-restart runs that supply training pairs")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--form", default="push", choices=["push", "pull"],
                    help="first-order kernel: push form (default) or the pull form of eq. kernel (its "
                         "divergence in closed form); the screened forms are push-form only")
    ap.add_argument("--operator", action="store_true",
                    help="predict with the stored operator (Sec. 10 offline/online split): built once per node "
                         "set inside the timed loop, applied every step; the roofline is the apply's HBM stream")
    ap.add_argument("--batch-forms", default="matrix", choices=["matrix", "tuned", "rule"],
                    help="batch64: each run's pairwise form -- the matrix-core form for every run (matrix, the "
                         "default), chosen per run by timing (tuned), or plain FP32 on the vector ALUs below "
                         "r = 32 (rule)")
    ap.add_argument("--e1-table", action="store_true",
                    help="the paper's large-scale test at its six sizes: time, RMSE and ME over --seeds runs of "
                         "1000 steps, beside the paper's table")
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--form-compare", action="store_true",
                    help="push form against the pull form on the r=2, r=10 and r=100 workloads over --seeds runs")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one 1 GiB copy + one yy_propagate, for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build benchmarks one GPU only; run with --gpus 1"}))
        sys.exit(2)

    args.prec_given = args.prec
    if args.prec is None:
        args.prec = "bf16x3g" if args.form == "pull" else ("fp32" if args.operator else "bf16x3p")
    if args.workload == "batch64":
        return main_batch(args)
    if args.e1_table:
        return main_e1_table(args)
    if args.form_compare:
        return main_form_compare(args)

    import numpy as np
    import torch

    from paper_2509_16896_amd import workloads as W

    if args.workload.startswith("paper_e1_r"):
        w = W.paper_e1(int(args.workload[len("paper_e1_r"):]))
        if args.prec_given is None and not args.operator and args.form == "push":
            args.prec = w.precision   # the plain FP32 form below r = 32
    else:
        w = {"cubic_r1000": W.cubic_r1000, "cubic_r100": W.cubic_r100}[args.workload]()
    if args.traffic_probe:
        w.K = 2
        traffic_probe(w, args.prec)
        return
    total = args.warmup + args.steps
    w.K = max(w.K, total + 1)
    xs, dys = W.simulate(w)
    log(f"[bench] workload {w.name}: r={w.r} n={w.n} scales={w.scales} prec={args.prec} "
        f"warmup={args.warmup} steps={args.steps} proposal={args.proposal}")
    prop_info, params = None, None
    if args.proposal == "learned":
        from paper_2509_16896_amd import proposal as PR

        t0 = time.perf_counter()
        X, MU, VAR = PR.collect_pairs(w, range(1000, 1000 + args.train_runs), prec=args.prec)
        params, losses = PR.train(w, X, MU, VAR, hidden=256, steps=args.train_steps, lr=1e-3,
                                  log_every=max(args.train_steps - 1, 1))
        prop_info = {"train_runs": args.train_runs, "pairs": int(X.shape[0]), "train_steps": args.train_steps,
                     "loss_first_last": [round(losses[0][1], 4), round(losses[-1][1], 4)],
                     "setup_s": round(time.perf_counter() - t0, 2)}
        log(f"[bench] proposal trained on {X.shape[0]} pairs in {prop_info['setup_s']} s, loss {losses}")
    f, k_last, elapsed, ms, launches = run_gpu(w, dys, args.prec, args.warmup, args.steps, proposal_params=params,
                                               form=args.form, operator=args.operator)
    if prop_info is not None:
        prop_info["used_fraction"] = round(int(f.used_count.item()) / max(f.restarts - 0, 1), 3)
    steps_s = args.steps / elapsed
    avg_kernel_s = (ms / 1e3) / max(launches, 1)
    mfma = args.prec != "fp32"
    method = alg_flops(w)
    alg, executed = method, method * EXEC_PER_ALG.get(args.prec, 1.0)
    screen = None
    kernel = "k_pair_mfma" if mfma else "k_pair_valu"
    basis = "2 n^2 r P: the method's products x.x and x.f for every pair"
    if args.prec in ("bf16x3s", "bf16x3p"):
        # the pairwise time is the screen plus the split pass over the flagged tiles
        from paper_2509_16896_amd import yy
        flagged, tiles = yy.yy_screen_count(f.ctx)
        screen = {"flagged_tiles": flagged, "tiles": tiles}
        alg, executed = screened_work(w, args.prec, flagged, tiles)
        sym = screen_pairs(w.n, args.prec, w.r) < float(w.n) * w.n
        kernel = ("k_tgt_bound, k_pair_prescreen_sym and k_sym_recheck" if sym else
                  "k_pair_prescreen" if args.prec == "bf16x3p" else "k_pair_screen") + \
            ", then k_pair_mfma (split form) on flagged tiles"
        basis = (f"the screen's x.x over the first {min(PRE_K, w.r)} coordinates for every pair it forms "
                 f"({'each pair of target blocks once: ' if sym else ''}{screen_pairs(w.n, args.prec, w.r):.6g} pairs), "
                 f"plus 2 r P per pair of the flagged tiles ({flagged} of {tiles})" if args.prec == "bf16x3p" else
                 f"the screen's x.x over all r coordinates for every pair, plus 2 r P per pair of the "
                 f"flagged tiles ({flagged} of {tiles})")
        log(f"[bench] screen flagged {flagged} of {tiles} tiles for the split form")
    achieved = alg / avg_kernel_s / 1e12
    peak = PEAK_TFLOPS[args.prec] if mfma else VALU_FP32_PEAK
    log(f"[bench] {steps_s:.3f} steps/s, pairwise kernels {1e3 * avg_kernel_s:.3f} ms per propagation "
        f"({launches} launches), {achieved:.1f} TFLOP/s on the executed work")
    roofline = {"bound": "mfma" if mfma else "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s"}
    roofline["frac"] = round(roofline["achieved"] / roofline["peak"], 4)
    roofline["traffic"] = recorded_traffic(args.prec) if args.workload == "cubic_r1000" else None
    roofline["work_basis"] = basis
    roofline["work_flop_per_launch"] = alg
    roofline["kernel"] = kernel
    roofline["kernel_ms"] = round(1e3 * avg_kernel_s, 3)
    if mfma:
        # matrix-core utilisation: executed products (3 BF16 products per split product) / peak
        roofline["mfma_exec_frac"] = round(executed / avg_kernel_s / 1e12 / peak, 4)
    # the method's work 2 n^2 r P per propagation, every pair formed: a dense evaluation at the peak
    # needs method / peak; the ratio to the measured time is the method-basis fraction (above 1 when
    # the screen rules pairs out -- it is no hardware rate)
    dense_at_peak_ms = method / (peak * 1e12) * 1e3
    roofline["method_work_flop_per_launch"] = method
    roofline["method_dense_at_peak_ms"] = round(dense_at_peak_ms, 4)
    roofline["frac_method_basis"] = round(dense_at_peak_ms / (1e3 * avg_kernel_s), 4)
    op_info = None
    if args.operator:
        # the online stage streams the stored exponents once: S n ld FP32 values, the n FP32 source
        # weights, and S n partial (max, sum) pairs written
        from paper_2509_16896_amd import yy
        nn, S, ebytes = yy.yy_operator_info(f.op)
        nbytes = ebytes + 4 * nn + 8 * S * nn
        gbs = nbytes / avg_kernel_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 2), "peak": 8000.0, "unit": "GB/s",
                    "frac": round(gbs / 8000.0, 4), "traffic": None,
                    "work_basis": "bytes per apply: S n ceil(n/64)*64 stored FP32 exponents + 4 n + 8 S n",
                    "work_bytes_per_launch": nbytes, "kernel": "k_op_apply", "kernel_ms": round(1e3 * avg_kernel_s, 4)}
        op_info = {"stored_bytes": ebytes, "builds_in_timed_steps": int(sum(
            1 for k in range(k_last - args.steps + 1, k_last + 1) if w.restart_every and k % w.restart_every == 1))}
        log(f"[bench] operator apply {1e3 * avg_kernel_s:.4f} ms, {gbs:.0f} GB/s of {nbytes / 1e6:.1f} MB")

    forms = {}
    if args.other_forms != "none":
        for p in [x for x in args.other_forms.split(",") if x and x != args.prec]:
            g, _, el3, ms3, l3 = run_gpu(w, dys, p, 1, 2)
            kms = ms3 / max(l3, 1)
            entry = {"kernel_ms": round(kms, 3), "steps_per_s": round(2 / el3, 4)}
            if p in ("bf16x3s", "bf16x3p"):
                from paper_2509_16896_amd import yy
                fl, tl = yy.yy_screen_count(g.ctx)
                a3, e3 = screened_work(w, p, fl, tl)
                entry.update(flagged_tiles=fl, tiles=tl)
            else:
                a3, e3 = method, method * EXEC_PER_ALG.get(p, 1.0)
                entry["method_tflops"] = round(method / (kms * 1e-3) / 1e12, 2)
                entry["frac_method"] = round(entry["method_tflops"] / PEAK_TFLOPS[p], 4)
            entry["executed_tflops"] = round(e3 / (kms * 1e-3) / 1e12, 2)
            entry["mfma_exec_frac"] = round(entry["executed_tflops"] / PEAK_TFLOPS[p], 4)
            forms[p] = entry
            g.close()
            log(f"[bench] form {p}: pairwise kernel {kms:.2f} ms")

    base = None
    if args.baseline_prec != "none" and args.baseline_prec != args.prec:
        g, _, el2, ms2, l2 = run_gpu(w, dys, args.baseline_prec, 1, args.baseline_steps)
        base = {"prec": args.baseline_prec, "steps_per_s": round(args.baseline_steps / el2, 4),
                "kernel_ms": round(ms2 / max(l2, 1), 3)}
        g.close()
        log(f"[bench] plain {args.baseline_prec}: {base['steps_per_s']} steps/s")
    # the same algorithm (every pair formed) against the plain FP32 form: pairwise-time ratios
    equal_alg = None
    if base is not None and forms:
        equal_alg = {p: round(base["kernel_ms"] / forms[p]["kernel_ms"], 3)
                     for p in ("bf16x3", "bf16x3g", "bf16x1") if p in forms}
    # second roofline record: the split form on every tile (the method's products for every pair)
    roofline_dense = None
    if DENSE_FORM in forms and args.workload == "cubic_r1000":
        d = forms[DENSE_FORM]
        roofline_dense = {"bound": "mfma", "achieved": d["method_tflops"], "peak": PEAK_TFLOPS[DENSE_FORM],
                          "unit": "TFLOP/s", "frac": d["frac_method"],
                          "traffic": recorded_traffic(DENSE_FORM),
                          "work_basis": "2 n^2 r P: the method's products x.x and x.f for every pair",
                          "kernel": "k_pair_mfma (BF16X3G split form, every tile)", "kernel_ms": d["kernel_ms"],
                          "mfma_exec_frac": d["mfma_exec_frac"]}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample of the step ...")
        cpu, sample = cpu_baseline(w, f, k_last, args.cpu_seconds, form=args.form)
        parity = sampled_parity(w, f, args.prec, sample)
        log(f"[bench] oracle {cpu['value']:.3g} steps/s on {cpu['cores']} threads; sampled rows max rel err {parity:.3g}")
    f.close()

    dtype = {"fp32": "f32", "fp32_mfma": "f32", "bf16x3": "bf16", "bf16x3g": "bf16", "bf16x3s": "bf16",
             "bf16x3p": "bf16", "bf16x1": "bf16"}[args.prec]
    line = {
        "metric": METRIC, "value": round(steps_s, 4), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "r": w.r, "n": w.n, "dt": w.dt, "scales": list(w.scales),
                   "restart_every": w.restart_every, "R": w.R, "precision": args.prec, "form": args.form,
                   "operator": args.operator},
        "propagation_tflops_executed": round(alg * args.steps / elapsed / 1e12, 3),
        "roofline": roofline,
        "roofline_dense": roofline_dense,
        "screen": screen,
        "plain_fp32": base,
        "vs_plain_fp32": None if base is None else round(steps_s / base["steps_per_s"], 3),
        "vs_plain_fp32_equal_algorithm_pairwise": equal_alg,
        "other_forms": forms or None,
        "proposal": prop_info,
        "operator": op_info,
        "sampled_row_max_rel_err": parity,
        "cpu_baseline": cpu,
    }
    if args.workload.startswith("paper_e1_r"):
        # the paper's runs take 1000 steps of this workload
        line["time_for_1000_steps_s"] = round(1000.0 / steps_s, 4)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
