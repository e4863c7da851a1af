"""Whole filter runs on the GPU against the FP64 oracle's filter (Sec. 2.2.2 procedure with the Sec. 6
local restart), every step, on the stored oracle results of ``tests/golden/make_filter_goldens.py``.

* cubic sensor r = 1000 with n = 4096, all 50 steps (the benchmarked workload with fewer nodes);
* cubic sensor r = 100, n = 16384, all 100 steps;
* six runs of the 64-run batch workload, all 100 steps, through the batched step;
* the six uneven runs of the batch tests, 8 steps, through the batched step;
* both batches also in BF16X3P with every run set to the split form on every tile (no screen).

Bars: the plain FP32 forms (direct differences, and the FP32 matrix-core form with exact near pairs)
match the posterior means to 1e-5 absolute at every step; the mixed-precision forms match them to 1e-3
absolute with the RMSE to the true path within 1 % of the oracle's (the RMSE and ME of Sec. 11).
"""
import os

import numpy as np
import pytest
import torch

from paper_2509_16896_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name, w):
    g = np.load(os.path.join(GOLDEN, f"filter_{name}.npz"))
    assert (int(g["r"]), int(g["n"]), int(g["K"]), float(g["dt"]), int(g["seed"])) == (w.r, w.n, w.K, w.dt, w.seed)
    return g


def _run(w, dys, prec):
    from paper_2509_16896_amd.filter import GpuFilter
    f = GpuFilter(w, prec=prec)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        torch.cuda.synchronize()
        return f.hist.cpu().numpy(), f.logZ_hist.cpu().numpy(), f.ess_hist.cpu().numpy()
    finally:
        f.close()


def _check(tag, means, logZ, xs, g, tol):
    ref = g["means"]
    err = float(np.max(np.abs(means - ref)))
    rg, ro = W.rmse(means, xs[1:]), W.rmse(ref, xs[1:])
    mg, mo = W.mean_error(means, xs[1:]), W.mean_error(ref, xs[1:])
    lz = float(np.max(np.abs(logZ - g["logZ"]) / np.maximum(1.0, np.abs(g["logZ"]))))
    print(f"{tag}: max |mean - oracle| = {err:.3g} (tol {tol}); RMSE {rg:.5f} vs oracle {ro:.5f}; "
          f"ME {mg:.5f} vs {mo:.5f}; max relative logZ difference {lz:.3g}", flush=True)
    assert np.all(np.isfinite(means))
    assert err <= tol
    assert abs(rg - ro) <= 0.01 * ro
    assert lz <= 1e-4


@pytest.mark.parametrize("prec,tol", [("bf16x3p", 1e-3), ("fp32", 1e-5), ("fp32_mfma", 1e-5)])
def test_cubic_r1000_n4096_all_steps(prec, tol):
    w = W.shrink(W.cubic_r1000(), n=4096, name="cubic_r1000_n4096")
    g = _golden("cubic_r1000_n4096", w)
    xs, dys = W.simulate(w)
    means, logZ, _ = _run(w, dys, prec)
    _check(f"r=1000 n=4096 K=50 [{prec}]", means, logZ, xs, g, tol)


@pytest.mark.parametrize("prec,tol", [("bf16x3p", 1e-3), ("bf16x3g", 1e-3), ("fp32", 1e-5)])
def test_cubic_r100_n16384_all_steps(prec, tol):
    w = W.cubic_r100()
    g = _golden("cubic_r100_n16384", w)
    xs, dys = W.simulate(w)
    means, logZ, _ = _run(w, dys, prec)
    _check(f"r=100 n=16384 K=100 [{prec}]", means, logZ, xs, g, tol)


def _batch_check(names, ws, prec, tol, every_tile=False):
    from paper_2509_16896_amd.batch import Batch
    sims = [W.simulate(w) for w in ws]
    bt = Batch(ws, [d for _, d in sims], prec=prec)
    try:
        if every_tile:
            # BF16X3P batch, every run with the split form on every tile (no screen)
            for q in range(len(ws)):
                bt.set_run_form(q, "bf16x3g")
        for _ in range(ws[0].K):
            bt.step()
        for q, (name, w) in enumerate(zip(names, ws)):
            res = bt.results(q)
            torch.cuda.synchronize()     # the copies run on the batch's own stream
            mean, lz, _ = (t.cpu().numpy() for t in res)
            form = bt.run_form(q)
            _check(f"batch {name} r={w.r} n={w.n} [{prec}, run form {form}]", mean, lz, sims[q][0],
                   _golden(name, w), tol)
    finally:
        bt.close()


BATCH64_RUNS = (21, 48, 3, 53, 2, 13)


@pytest.mark.parametrize("prec,tol,every_tile", [("bf16x3p", 1e-3, False), ("bf16x3p", 1e-3, True),
                                                 ("fp32_mfma", 1e-5, False)])
def test_batch64_sample_runs_all_steps(prec, tol, every_tile):
    runs = W.batch_runs(64)
    _batch_check([f"batch64_run{b}" for b in BATCH64_RUNS], [runs[b] for b in BATCH64_RUNS], prec, tol,
                 every_tile)


@pytest.mark.parametrize("prec,tol,every_tile", [("bf16x3p", 1e-3, False), ("bf16x3p", 1e-3, True),
                                                 ("bf16x3g", 1e-3, False), ("fp32_mfma", 1e-5, False)])
def test_batch6_uneven_runs(prec, tol, every_tile):
    shapes = ((10, 2048), (33, 1024), (64, 4096), (100, 2048), (150, 1024), (200, 8192))
    ws = []
    for b, (r, n) in enumerate(shapes):
        ws.append(W.Workload(f"batch_r{r}_n{n}", r=r, n=n, dt=0.01, K=8, drift=W.F_COS, obs=W.H_CUBE, q=0.09,
                             rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3 + 0.1 * b, restart_every=2, R=0.3,
                             seed=b + 1))
    _batch_check([f"batch6_run{b}" for b in range(6)], ws, prec, tol, every_tile)
