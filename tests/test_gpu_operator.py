"""The stored operator (Sec. 10 offline / online split, Sec. 4.2 steps 2-3 and 5, Sec. 9 log domain):
yy_operator_build stores every kernel value of a node set; yy_operator_apply gives the prediction.

Checked against the oracle's prediction (the definition) at the FP32 parity bar of the recomputing
path (1e-5 on normalised log-densities), and against yy_propagate's plain FP32 form (the same
arithmetic up to summation order): push and pull forms, one to four scales, boundary nodes, sparse
weights, general noise; several weight vectors on one build; a rebuild in place on a new node set and
on a larger one; the memory it reports; whole filter runs predicting with the operator against the
oracle's filter.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import compare_logw, dev, host, next_version
from oracle import filter as ofilter
from paper_2509_16896_amd import workloads as W

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")


@pytest.fixture(scope="module")
def ctx():
    c = yy.yy_create(0, torch.cuda.current_stream())
    yield c
    yy.yy_destroy(c)


CASES = {
    "cubic_r2_n1024_s12": dict(r=2, n=1024, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.01, half=4.0, seed=0),
    "linear_r10_n4000_s1": dict(r=10, n=4000, drift=oracle.F_LINEAR, scales=(1.0,), q=0.1, dt=0.01, half=0.75, seed=2),
    "sinmix_r10_n100_s124": dict(r=10, n=100, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0, dt=0.01,
                                 half=0.3, seed=7),
    "cos_r64_n513_s124_unscrambled": dict(r=64, n=513, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09, dt=0.005,
                                          half=0.3, seed=11, scramble=False),
    "zero_r3_n65_sparse_s12": dict(r=3, n=65, drift=oracle.F_ZERO, scales=(1.0, 2.0), q=1.0, dt=0.05, half=1.0,
                                   seed=5, lw_kind="sparse"),
    "cos_r65_n300_s1248": dict(r=65, n=300, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0, 8.0), q=0.2, dt=0.02,
                               half=0.4, seed=21),
    "sinmix_r1000_n500_s124": dict(r=1000, n=500, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0,
                                   dt=0.01, half=0.3, seed=8),
}


def _inputs(r, n, drift, scales, q, dt, half, seed, scramble=True, lw_kind="random"):
    k = np.arange(r)
    lo, hi = -half + 0.01 * np.sin(k), half + 0.02 * np.cos(k)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, scramble, seed), lo, hi)
    A = W.linear_drift_matrix(r, 0) if drift == oracle.F_LINEAR else None
    return lo, hi, x, A


def _weights(n, x, lo, hi, half, seed, lw_kind="random"):
    rng = np.random.default_rng(seed)
    if lw_kind == "random":
        return -3.0 * rng.random(n) - 0.5 * np.sum(((x - 0.5 * (lo + hi)) / half) ** 2, axis=1)
    lw = np.full(n, -np.inf)
    lw[rng.integers(0, n, 3)] = rng.standard_normal(3)
    return lw


@pytest.mark.parametrize("form", ["push", "pull"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_operator_apply_equals_the_prediction(ctx, name, form):
    kw = CASES[name]
    r, n = kw["r"], kw["n"]
    lo, hi, x, A = _inputs(**kw)
    om = oracle.OModel(r, r, kw["drift"], A, oracle.H_IDENTITY, None, 0.0, kw["q"], 1.0)
    gm = yy.Model(r, r, kw["drift"], A, yy.YY_H_IDENTITY, None, 0.0, kw["q"], 1.0)
    sc = yy.Scales(kw["scales"], form=form)
    c = oracle.kernel_coefficients(kw["scales"])
    oform = oracle.FORM_PULL if form == "pull" else oracle.FORM_PUSH
    xd, lod, hid = dev(x.ravel()), dev(lo), dev(hi)
    op = yy.yy_operator_build(ctx, gm, sc, n, xd, next_version(), lod, hid, kw["dt"])
    try:
        nn, S, nbytes = yy.yy_operator_info(op)
        assert (nn, S, nbytes) == (n, len(kw["scales"]), len(kw["scales"]) * n * (((n + 63) // 64) * 64) * 4)
        # several weight vectors through one build
        for t in range(3):
            lw = _weights(n, x, lo, hi, kw["half"], kw["seed"] + 100 * t, kw.get("lw_kind", "random"))
            ref, _ = oracle.propagate_ex(om, kw["scales"], c, x, lo, hi, kw["dt"], lw, form=oform)
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            yy.yy_operator_apply(op, dev(lw), out)
            got = host(out)
            worst, cnt = compare_logw(got, ref, 1e-5)
            print(f"operator {name} [{form}] weights {t}: worst err/allowed = {worst:.3g} over {cnt} nodes", flush=True)
            assert worst <= 1.0
            assert np.array_equal(np.isfinite(got), np.isfinite(ref))
            # the recomputing plain FP32 form: the same arithmetic up to the order of the sums
            rec = torch.empty(n, dtype=torch.float64, device="cuda")
            yy.yy_propagate(ctx, gm, sc, "fp32", n, xd, next_version(), lod, hid, kw["dt"], dev(lw), rec)
            rec = host(rec)
            f = np.isfinite(rec)
            assert np.array_equal(f, np.isfinite(got))
            assert np.max(np.abs(got[f] - rec[f]) / np.maximum(1.0, np.abs(rec[f]))) < 2e-6
    finally:
        yy.yy_operator_destroy(op)


def test_operator_rebuild_in_place_and_larger(ctx):
    r, q, dt, half = 6, 0.5, 0.02, 0.7
    om = oracle.OModel(r, r, oracle.F_COS, None, oracle.H_IDENTITY, None, 0.0, q, 1.0)
    gm = yy.Model(r, r, yy.YY_F_COS, None, yy.YY_H_IDENTITY, None, 0.0, q, 1.0)
    s = (1.0, 2.0, 4.0)
    c = oracle.kernel_coefficients(s)
    op = None
    try:
        for n, seed in ((700, 1), (700, 2), (1500, 3)):   # same size, new nodes; then a larger set
            lo, hi = -half * np.ones(r), half * np.ones(r)
            x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, True, seed), lo, hi)
            op = yy.yy_operator_build(ctx, gm, yy.Scales(s), n, dev(x.ravel()), next_version(), dev(lo), dev(hi),
                                      dt, op)
            lw = _weights(n, x, lo, hi, half, seed)
            ref, _ = oracle.propagate(om, s, c, x, lo, hi, dt, lw)
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            yy.yy_operator_apply(op, dev(lw), out)
            worst, _ = compare_logw(host(out), ref, 1e-5)
            assert worst <= 1.0, (n, seed)
    finally:
        if op is not None:
            yy.yy_operator_destroy(op)


def test_operator_with_general_noise(ctx):
    r, n, dt = 8, 900, 0.02
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((r, r)))
    U = Q @ np.diag(np.sqrt(np.r_[0.2 + 0.3 * rng.random(r - 2), 0.0, 0.0]))
    ap, logdet, _ = oracle.noise_pinv(U)
    lo, hi = -0.5 * np.ones(r), 0.5 * np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, True, 3), lo, hi)
    lw = _weights(n, x, lo, hi, 0.5, 3)
    s = (1.0, 2.0)
    om = oracle.OModel(r, r, oracle.F_COS, None, oracle.H_IDENTITY, None, 0.0, 1.0, 1.0)
    ref, _ = oracle.propagate_ex(om, s, oracle.kernel_coefficients(s), x, lo, hi, dt, lw, apinv=ap, logdet_a=logdet)
    nz = yy.yy_noise_create(ctx, r, U, r, None)
    op = None
    try:
        gm = yy.Model(r, r, yy.YY_F_COS, None, yy.YY_H_IDENTITY, None, 0.0, 1.0, 1.0, noise=nz)
        op = yy.yy_operator_build(ctx, gm, yy.Scales(s), n, dev(x.ravel()), next_version(), dev(lo), dev(hi), dt)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        yy.yy_operator_apply(op, dev(lw), out)
        worst, _ = compare_logw(host(out), ref, 1e-5)
        assert worst <= 1.0
    finally:
        if op is not None:
            yy.yy_operator_destroy(op)
        yy.yy_noise_destroy(nz)


FILTERS = {
    "cubic_r2_n1024_K100_full": W.cubic_r2(),
    "linear_r10_n2048_K10_restart": W.shrink(W.linear_r10(), n=2048, K=10),
    "paper_e1_r10_n100_K20": W.shrink(W.paper_e1(10), K=20),
    "cubic_r20_n1024_K6_restart_s124": W.shrink(W.cubic_r100(), r=20, n=1024, K=6),
}


@pytest.mark.parametrize("name", sorted(FILTERS))
def test_filter_with_the_operator_matches_oracle(name):
    from paper_2509_16896_amd.filter import GpuFilter
    w = FILTERS[name]
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    f = GpuFilter(w, prec="fp32", operator=True)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        torch.cuda.synchronize()
        got = f.hist.cpu().numpy()
    finally:
        f.close()
    err = float(np.max(np.abs(got - ref["means"])))
    print(f"operator filter {name}: max |mean - oracle| = {err:.3g}", flush=True)
    assert err <= 1e-5
