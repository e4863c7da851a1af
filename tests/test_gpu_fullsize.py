"""Parity at the workloads' full sizes.

* Cubic sensor r=1000, n=65536 (the benchmarked workload, in the launch
  configuration the benchmark times): the GPU's propagation of a filter state
  against the oracle on sampled target rows, which it computes one by one.
* Linear-Gaussian r=10, n=4096, 200 steps with restarts: the whole GPU filter
  against the oracle's filter, and its RMSE beside the Kalman filter's.
* Cubic sensor r=100, n=16384, a few steps with a restart: the chosen
  mixed-precision form and the FP32 form against the oracle's filter.
* Cubic sensor r=1000, n=65536, four steps with two restarts: the chosen form's
  posterior means against the plain FP32 form's (the oracle's filter takes
  minutes per step at this size; the FP32 form matches it to 1e-5 on the
  smaller workloads above); and all 50 steps in the chosen form against the
  plain FP32 matrix-core form, with their RMSEs to the true path.
"""
import numpy as np
import pytest
import torch
from scipy.special import logsumexp

import oracle
from oracle import filter as ofilter
from oracle import kalman
from paper_2509_16896_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu_filter(w, dys, prec, steps):
    from paper_2509_16896_amd.filter import GpuFilter
    f = GpuFilter(w, prec=prec)
    f.set_observations(dys)
    f.init()
    for k in range(1, steps + 1):
        f.step(k)
    torch.cuda.synchronize()
    return f


@pytest.mark.parametrize("prec,tol", [("bf16x3p", 1e-5), ("bf16x3s", 1e-5), ("bf16x3g", 1e-5), ("bf16x3", 1e-5), ("bf16x1", 1e-5),
                                      ("fp32_mfma", 1e-5)])
def test_cubic_r1000_n65536_sampled_rows(prec, tol):
    from paper_2509_16896_amd import yy
    w = W.cubic_r1000()
    xs, dys = W.simulate(w)
    f = _gpu_filter(w, dys, prec, 3)   # a restart at step 2, then one more step
    try:
        out = torch.empty(w.n, dtype=torch.float64, device="cuda")
        yy.yy_propagate(f.ctx, f.model, f.scales, prec, w.n, f.x, f.version, f.lo, f.hi, w.dt, f.lw[f.cur], out)
        got = out.cpu().numpy()
        x = f.x.cpu().numpy().reshape(w.n, w.r)
        lw = f.lw[f.cur].cpu().numpy()
        lo, hi = f.lo.cpu().numpy(), f.hi.cpu().numpy()
    finally:
        f.close()
    rng = np.random.default_rng(7)
    # the heaviest node, the lightest finite one, the first and last rows (ragged tail) and random rows
    fin = np.flatnonzero(np.isfinite(lw))
    rows = np.unique(np.concatenate([[int(np.argmax(lw)), int(fin[np.argmin(lw[fin])]), 0, w.n - 1],
                                     rng.choice(w.n, 20, replace=False)]))
    s = np.asarray(w.scales)
    ref, _ = oracle.propagate_rows(ofilter.model_of(w), s, oracle.kernel_coefficients(s), x, lo, hi, w.dt, lw, rows)
    z = logsumexp(got[np.isfinite(got)])
    g = got[rows]
    assert np.array_equal(np.isfinite(g), np.isfinite(ref))
    ok = np.isfinite(ref)
    err = np.abs(g[ok] - ref[ok]) / np.maximum(1.0, np.abs(ref[ok] - z))
    print(f"{prec}: {ok.sum()} rows, max relative error {err.max():.3g}")
    assert err.max() <= tol


def test_linear_r10_full_run_and_kalman():
    w = W.linear_r10()
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    f = _gpu_filter(w, dys, "fp32", w.K)
    try:
        means = f.hist.cpu().numpy()
    finally:
        f.close()
    err = np.max(np.abs(means - ref["means"]))
    m_kf, _ = kalman.kalman_filter(w.A, np.eye(w.r), w.q, w.rho2, w.dt, dys, np.zeros(w.r), np.eye(w.r))
    ratio = W.rmse(means, xs[1:]) / W.rmse(m_kf, xs[1:])
    print(f"max |mean - oracle| = {err:.3g}; RMSE / RMSE(Kalman) = {ratio:.4f}")
    assert err <= 1e-5
    # statistical: the restarted filter on 4096 quasi-random nodes in 10 dimensions (about 2.3
    # nodes per coordinate) stays within 40 % of the exact linear-Gaussian filter's RMSE
    # (1.25 measured; the oracle's own filter gives the same, its means agree to 1e-5)
    assert 0.9 <= ratio <= 1.4


def test_cubic_r100_n16384_short_run():
    w = W.shrink(W.cubic_r100(), K=3)
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    for prec, tol in [("bf16x3p", 1e-3), ("bf16x3s", 1e-3), ("bf16x3g", 1e-3), ("fp32", 1e-5)]:
        f = _gpu_filter(w, dys, prec, w.K)
        try:
            means = f.hist.cpu().numpy()
        finally:
            f.close()
        err = np.max(np.abs(means - ref["means"]))
        print(f"{prec}: max |mean - oracle| = {err:.3g}")
        assert err <= tol


@pytest.mark.parametrize("prec", ["bf16x3p", "bf16x3s"])
def test_cubic_r1000_n65536_chosen_form_means(prec):
    w = W.shrink(W.cubic_r1000(), K=4)
    xs, dys = W.simulate(w)
    fs = _gpu_filter(w, dys, prec, w.K)
    try:
        got = fs.hist.cpu().numpy()
    finally:
        fs.close()
    fp = _gpu_filter(w, dys, "fp32", w.K)
    try:
        ref = fp.hist.cpu().numpy()
    finally:
        fp.close()
    err = np.max(np.abs(got - ref))
    print(f"r=1000, n=65536, 4 steps: max |mean({prec}) - mean(fp32)| = {err:.3g}")
    assert np.all(np.isfinite(got))
    assert err <= 1e-3


def test_cubic_r1000_n65536_full_run_chosen_form():
    """All 50 steps (24 restarts, learned proposal off) in the chosen form against the plain FP32 form:
    the posterior means agree to 1e-3 at every step, and so do their RMSEs to the true path."""
    w = W.cubic_r1000()
    xs, dys = W.simulate(w)
    out = {}
    for prec in ("bf16x3p", "fp32_mfma"):
        f = _gpu_filter(w, dys, prec, w.K)
        try:
            out[prec] = f.hist.cpu().numpy()
        finally:
            f.close()
    got, ref = out["bf16x3p"], out["fp32_mfma"]
    err = float(np.max(np.abs(got - ref)))
    rg, rr = W.rmse(got, xs[1:]), W.rmse(ref, xs[1:])
    print(f"r=1000, n=65536, {w.K} steps: max |mean(bf16x3p) - mean(fp32_mfma)| = {err:.3g}; "
          f"RMSE to truth {rg:.4f} against {rr:.4f}")
    assert np.all(np.isfinite(got))
    assert err <= 1e-3
    assert abs(rg - rr) <= 1e-3 * max(rr, 1e-12) + 1e-6
