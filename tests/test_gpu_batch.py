"""The batched filter (one pairwise launch for all runs per step), its HIP graph
replay and the autotuners, against single-run filters through the same C ABI."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import host

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")
from paper_2509_16896_amd import workloads as W  # noqa: E402
from paper_2509_16896_amd.batch import Batch  # noqa: E402
from paper_2509_16896_amd.filter import GpuFilter  # noqa: E402

# uneven runs: r across the matrix-core K steps, n powers of two (a ragged tile
# count for the smallest), restart every 2 steps
SHAPES = [(10, 2048), (33, 1024), (64, 4096), (100, 2048), (150, 1024), (200, 8192)]


def _workloads(K=8, shapes=SHAPES):
    out = []
    for b, (r, n) in enumerate(shapes):
        out.append(W.Workload(f"batch_r{r}_n{n}", r=r, n=n, dt=0.01, K=K, drift=W.F_COS, obs=W.H_CUBE, q=0.09,
                              rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3 + 0.1 * b, restart_every=2, R=0.3,
                              seed=b + 1))
    return out


def _single(w, dys, prec):
    # the batched step makes the correction and the normalisation as two calls
    f = GpuFilter(w, prec=prec, one_pass=False)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        return host(f.hist), host(f.logZ_hist), host(f.ess_hist)
    finally:
        f.close()


@pytest.mark.parametrize("small_r", ["matrix", "fp32"])
@pytest.mark.parametrize("prec", ["bf16x3g", "bf16x3s", "bf16x3p", "fp32_mfma"])
def test_batch_matches_single_runs_exactly(prec, small_r):
    """Every run against the single-run filter in the run's form: all runs in the batch's matrix-core
    form (the default, "matrix"), or the runs below r = 32 set to the plain FP32 form ("fp32")."""
    ws = _workloads()
    dys = [W.simulate(w)[1] for w in ws]
    bt = Batch(ws, dys, prec=prec, max_split=16)
    try:
        for q, w in enumerate(ws):
            assert bt.run_form(q) == prec
            if small_r == "fp32" and w.r < 32:
                bt.set_run_form(q, "fp32")
                assert bt.run_form(q) == "fp32"
        for _ in range(ws[0].K):
            bt.step()
        assert bt.k == ws[0].K
        for q, w in enumerate(ws):
            mean, lz, ess = (host(t) for t in bt.results(q))
            ref = _single(w, dys[q], bt.run_form(q))
            assert np.array_equal(mean, ref[0]), w.name
            assert np.array_equal(lz, ref[1]), w.name
            assert np.array_equal(ess, ref[2]), w.name
            assert np.all(np.isfinite(mean))
            if prec in ("bf16x3s", "bf16x3p") and bt.run_form(q) == prec:
                flagged, tiles = bt.screen_count(q)
                assert tiles == ((w.n + 255) // 256) * ((w.n + 127) // 128) and 0 <= flagged <= tiles
    finally:
        bt.close()


def test_batch_symmetric_screen_matches_single_runs():
    """Runs of more than 32 target blocks (n > 8192, ragged last blocks) take the symmetric screen in
    the batched step too, beside runs with the one-sided screen: bit for bit the single-run filter's
    results, with the flags of every screen within range."""
    shapes = [(64, 12000), (33, 9000), (100, 2048), (20, 8500)]
    ws = _workloads(K=6, shapes=shapes)
    dys = [W.simulate(w)[1] for w in ws]
    bt = Batch(ws, dys, prec="bf16x3p", max_split=16)
    try:
        for _ in range(ws[0].K):
            bt.step()
        for q, w in enumerate(ws):
            mean, lz, ess = (host(t) for t in bt.results(q))
            ref = _single(w, dys[q], "bf16x3p")
            assert np.array_equal(mean, ref[0]), w.name
            assert np.array_equal(lz, ref[1]), w.name
            assert np.array_equal(ess, ref[2]), w.name
            assert np.all(np.isfinite(mean))
            flagged, tiles = bt.screen_count(q)
            assert tiles == ((w.n + 255) // 256) * ((w.n + 127) // 128) and 0 <= flagged <= tiles
            print(f"{w.name}: flagged {flagged} of {tiles} tiles in the last step")
    finally:
        bt.close()


@pytest.mark.parametrize("prec", ["bf16x3g", "bf16x3s", "bf16x3p"])
def test_graph_replay_equals_eager_steps(prec):
    ws = _workloads(K=10)
    dys = [W.simulate(w)[1] for w in ws]
    a = Batch(ws, dys, prec=prec)
    g = Batch(ws, dys, prec=prec)
    try:
        for _ in range(10):
            a.step()
        ref = [[host(t) for t in a.results(q)] for q in range(len(ws))]
        for rep in range(2):   # the second launch reuses the captured graph
            g.reset()
            g.step()
            g.step()
            g.run_graph(10)
            assert g.k == 10
            torch.cuda.synchronize()
            for q in range(len(ws)):
                got = [host(t) for t in g.results(q)]
                for x, y in zip(got, ref[q]):
                    assert np.array_equal(x, y), (rep, q)
        # eager work between replays, then a third replay
        g.reset()
        g.step()
        g.step()
        _ = torch.ones(1000, device="cuda").sum().item()
        g.run_graph(10)
        for q in range(len(ws)):
            assert np.array_equal(host(g.results(q)[0]), ref[q][0])
    finally:
        a.close()
        g.close()


def test_graph_from_step_zero_with_odd_end():
    ws = _workloads(K=7)
    dys = [W.simulate(w)[1] for w in ws]
    a = Batch(ws, dys)
    g = Batch(ws, dys)
    try:
        for _ in range(7):
            a.step()
        g.run_graph(7)          # three graph launches of two steps, then one eager step
        assert g.k == 7
        with pytest.raises(yy.YYError):
            g.step()            # all K steps taken
        for q in range(len(ws)):
            for x, y in zip(g.results(q), a.results(q)):
                assert np.array_equal(host(x), host(y)), q
    finally:
        a.close()
        g.close()


def test_batch_tuner_keeps_results():
    """The tuner picks each run's form (matrix cores or vector ALUs) and the source splits; every run then
    matches the single-run filter in its chosen form (another split count changes only the summation
    order of the partial sums)."""
    ws = _workloads(K=6)
    dys = [W.simulate(w)[1] for w in ws]
    b = Batch(ws, dys, prec="bf16x3g")
    try:
        best = b.tune(reps=2, forms=True)
        assert best in (1, 2, 4, 8, 16, 32, 64)
        forms = [b.run_form(q) for q in range(len(ws))]
        print("tuned forms:", list(zip([w.r for w in ws], [w.n for w in ws], forms)))
        assert all(f in ("bf16x3g", "fp32") for f in forms)
        for _ in range(6):
            b.step()
        for q, w in enumerate(ws):
            mean = host(b.results(q)[0])
            ref = _single(w, dys[q], forms[q])[0]
            assert np.allclose(mean, ref, rtol=1e-9, atol=1e-9), w.name
    finally:
        b.close()


def test_batch_run_form_arguments():
    ws = _workloads(K=2)
    dys = [W.simulate(w)[1] for w in ws]
    b = Batch(ws, dys, prec="bf16x3p")
    s = Batch(ws[:2], dys[:2], prec="bf16x3s")
    try:
        with pytest.raises(yy.YYError):
            b.set_run_form(1, "bf16x1")         # neither the batch's form, fp32 nor (BF16X3P) bf16x3g
        with pytest.raises(yy.YYError):
            s.set_run_form(1, "bf16x3g")        # the split form on every tile only in a BF16X3P batch
        b.set_run_form(1, "bf16x3g")
        assert b.run_form(1) == "bf16x3g"
        b.set_run_form(1, "bf16x3p")
        assert b.run_form(1) == "bf16x3p"
        with pytest.raises(yy.YYError):
            b.run_form(len(ws))
        b.set_run_form(2, "fp32")               # r = 64 on the vector ALUs
        assert b.run_form(2) == "fp32"
        b.step()
        b.step()
        ref = _single(ws[2], dys[2], "fp32")
        assert np.array_equal(host(b.results(2)[0]), ref[0])
    finally:
        b.close()
        s.close()


# runs whose screen spans 32 coordinates (r <= 32) beside screened runs, one of them with the
# symmetric screen (n > 8192, r > 32) and ragged last target blocks
DENSE_SHAPES = [(10, 2048), (20, 8500), (24, 4096), (64, 4096), (33, 9000), (32, 1000)]


def test_batch_split_on_every_tile_runs():
    """Runs of a BF16X3P batch set to BF16X3G skip the screen and take the split form on every tile in
    BF16X3P's order: each flags every tile, and its results equal the single-run BF16X3P filter's up to
    the pairs that filter's screen drops (more than 2^-80 below their row's floor, so nothing at FP64
    rounding of the means here); the screened runs beside them stay bit for bit the single-run
    filter's.  The graph-replayed batch repeats the eager one exactly (the flags are set once, at the
    batch's build)."""
    ws = _workloads(K=6, shapes=DENSE_SHAPES)
    dys = [W.simulate(w)[1] for w in ws]
    dense = [q for q, w in enumerate(ws) if w.r <= 32]
    a = Batch(ws, dys, prec="bf16x3p", max_split=16)
    g = Batch(ws, dys, prec="bf16x3p", max_split=16)
    try:
        for bt in (a, g):
            for q in dense:
                bt.set_run_form(q, "bf16x3g")
        for _ in range(ws[0].K):
            a.step()
        g.step()
        g.step()
        g.run_graph(ws[0].K)
        for q, w in enumerate(ws):
            mean, lz, ess = (host(t) for t in a.results(q))
            for x, y in zip((mean, lz, ess), (host(t) for t in g.results(q))):
                assert np.array_equal(x, y), w.name
            ref = _single(w, dys[q], "bf16x3p")
            flagged, tiles = a.screen_count(q)
            assert tiles == ((w.n + 255) // 256) * ((w.n + 127) // 128)
            assert np.all(np.isfinite(mean))
            if q in dense:
                assert a.run_form(q) == "bf16x3g" and flagged == tiles, w.name
                dm = float(np.max(np.abs(mean - ref[0])))
                print(f"{w.name}: every tile; |mean - single-run BF16X3P| <= {dm:.3g}")
                assert np.allclose(mean, ref[0], rtol=0, atol=1e-12), w.name
                assert np.allclose(lz, ref[1], rtol=1e-12, atol=1e-12), w.name
                assert np.allclose(ess, ref[2], rtol=1e-12, atol=0), w.name
            else:
                assert np.array_equal(mean, ref[0]), w.name
                assert np.array_equal(lz, ref[1]), w.name
                assert np.array_equal(ess, ref[2]), w.name
    finally:
        a.close()
        g.close()


def test_batch_tuner_screen_or_every_tile():
    """The tuner's second search (BF16X3P batches): each run keeps its screen or takes the split form
    on every tile, whichever its single-run call runs faster; every run then matches the single-run
    BF16X3P filter (another split count changes only the summation order of the partial sums)."""
    ws = _workloads(K=6, shapes=DENSE_SHAPES)
    dys = [W.simulate(w)[1] for w in ws]
    b = Batch(ws, dys, prec="bf16x3p")
    try:
        for _ in range(2):
            b.step()
        best = b.tune(reps=2, dense=True)
        assert best in (1, 2, 4, 8, 16, 32, 64)
        forms = [b.run_form(q) for q in range(len(ws))]
        print("tuned forms:", list(zip([w.r for w in ws], [w.n for w in ws], forms)))
        assert all(f in ("bf16x3p", "bf16x3g") for f in forms)
        b.reset()
        for _ in range(6):
            b.step()
        for q, w in enumerate(ws):
            mean = host(b.results(q)[0])
            ref = _single(w, dys[q], "bf16x3p")[0]
            assert np.allclose(mean, ref, rtol=1e-9, atol=1e-9), w.name
    finally:
        b.close()


def test_single_run_tuner_table():
    w = dataclasses.replace(_workloads()[2], K=3)
    xs, dys = W.simulate(w)
    ref = _single(w, dys, "bf16x3g")
    f = GpuFilter(w, prec="bf16x3g")
    try:
        best = yy.yy_tune(f.ctx, [(w.r, w.n), (128, 16384)], f.scales, "bf16x3g", reps=2)
        assert all(v in (1, 2, 4, 8, 16, 32, 64, 128, 256) for v in best)
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        assert np.allclose(host(f.hist), ref[0], rtol=1e-9, atol=1e-9)
    finally:
        f.close()
