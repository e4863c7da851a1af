"""The pull-form kernel (Sec. 4.1, Theorem thm:1storderkernel, eq. kernel) on the GPU against the oracle.

* One prediction: the vector-ALU form and every matrix-core form that supports the pull form, against
  the oracle's pull form at 1e-5 on normalised log-densities (the parity metric of the push form), with
  the divergence in closed form and by complex step (Sec. 8); the single-node raw value (constants and
  the divergence factor); the screened forms are refused.
* Whole filter runs with the pull form against the oracle's filter with the pull form.
* Pull against push on the cubic-sensor and linear-Gaussian workloads: both forms are first-order
  consistent approximations of the same operator, so their filters' errors to the true path agree
  (statistical; printed beside each other).
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


def _case(r, n, drift, scales, q, dt, half, seed, div=oracle.DIV_CLOSED, scramble=True, lw_kind="random"):
    k = np.arange(r)
    lo, hi = -half + 0.01 * np.sin(k), half + 0.02 * np.cos(k)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, scramble, seed), lo, hi)
    rng = np.random.default_rng(seed)
    if lw_kind == "random":
        lw = -3.0 * rng.random(n) - 0.5 * np.sum(((x - 0.5 * (lo + hi)) / half) ** 2, axis=1)
    else:
        lw = np.full(n, -np.inf)
        lw[rng.integers(0, n, 3)] = rng.standard_normal(3)
    A = W.linear_drift_matrix(r, 0) if drift == oracle.F_LINEAR else None
    om = oracle.OModel(r, r, drift, A, oracle.H_IDENTITY, None, 0.0, q, 1.0)
    c = oracle.kernel_coefficients(scales)
    ref, ncl = oracle.propagate_ex(om, scales, c, x, lo, hi, dt, lw, form=oracle.FORM_PULL, div_mode=div)
    gm = yy.Model(r, r, drift, A, yy.YY_H_IDENTITY, None, 0.0, q, 1.0)
    return dict(lo=lo, hi=hi, x=x, lw=lw, ref=ref, gm=gm, scales=scales, dt=dt, n=n, r=r, div=div)


def _gpu(ctx, case, prec, form="pull"):
    n = case["n"]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    yy.yy_propagate(ctx, case["gm"], yy.Scales(case["scales"], form=form, div=case["div"]), prec, n,
                    dev(case["x"].ravel()), next_version(), dev(case["lo"]), dev(case["hi"]), case["dt"],
                    dev(case["lw"]), out)
    return host(out)


CASES = {
    "cubic_r2_n1024_s12": dict(r=2, n=1024, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.01, half=4.0, seed=0),
    "linear_r10_n2048_s1": dict(r=10, n=2048, drift=oracle.F_LINEAR, scales=(1.0,), q=0.1, dt=0.01, half=0.75,
                                seed=2),
    "sinmix_r10_n100_s124_cstep": dict(r=10, n=100, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0,
                                       dt=0.01, half=0.3, seed=7, div=oracle.DIV_COMPLEX_STEP),
    "zero_r3_n65_sparse": dict(r=3, n=65, drift=oracle.F_ZERO, scales=(1.0, 2.0), q=1.0, dt=0.05, half=1.0, seed=5,
                               lw_kind="sparse"),
    "cos_r64_n512_s124": dict(r=64, n=512, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09, dt=0.005, half=0.3,
                              seed=11),
    "cos_r100_n1000_ragged_s124_cstep": dict(r=100, n=1000, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09,
                                             dt=0.005, half=0.3, seed=12, div=oracle.DIV_COMPLEX_STEP),
    "sinmix_r50_n300_s124": dict(r=50, n=300, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0, dt=0.01,
                                 half=0.3, seed=13),
    "linear_r128_n2048_s12": dict(r=128, n=2048, drift=oracle.F_LINEAR, scales=(1.0, 2.0), q=0.1, dt=0.01, half=0.4,
                                  seed=14),
    "cos_r40_n1024_dense_near": dict(r=40, n=1024, drift=oracle.F_COS, scales=(1.0,), q=2.0, dt=0.05, half=0.25,
                                     seed=15),
    "cos_r64_n512_unscrambled_boundary": dict(r=64, n=512, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09,
                                              dt=0.005, half=0.3, seed=17, scramble=False),
    "cos_r65_n300_s1248": dict(r=65, n=300, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0, 8.0), q=0.2, dt=0.02,
                               half=0.4, seed=21),
    "cos_r1000_n600_s124": dict(r=1000, n=600, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09, dt=0.005,
                                half=0.3, seed=24),
}


@pytest.mark.parametrize("prec", ["fp32", "fp32_mfma", "bf16x3", "bf16x3g", "bf16x1"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_pull_propagate_parity(ctx, name, prec):
    case = _case(**CASES[name])
    got = _gpu(ctx, case, prec)
    worst, cnt = compare_logw(got, case["ref"], 1e-5)
    print(f"pull {name} [{prec}]: worst err/allowed = {worst:.3g} over {cnt} nodes", flush=True)
    assert worst <= 1.0
    bnd = oracle.is_boundary(case["x"], case["lo"], case["hi"])
    assert np.all(np.isneginf(got[bnd]))
    assert np.array_equal(np.isfinite(got), np.isfinite(case["ref"]))


@pytest.mark.parametrize("prec", ["fp32", "fp32_mfma", "bf16x3", "bf16x3g", "bf16x1"])
def test_pull_single_node_raw_value(ctx, prec):
    """One node: the raw value is the signed combination of the self-pair densities with the divergence
    factor exp(-tau_s div f(x)) -- constants included."""
    for r in (1, 40, 200):
        case = _case(r, 1, oracle.F_COS, (1.0, 2.0, 4.0), 0.09, 0.005, 0.3, 30 + r)
        got = _gpu(ctx, case, prec)
        ref = case["ref"]
        assert np.isfinite(ref[0]) == np.isfinite(got[0])
        if np.isfinite(ref[0]):
            assert abs(got[0] - ref[0]) <= 1e-5 * max(1.0, abs(ref[0])), (r, got[0], ref[0])


def test_pull_divergence_modes_agree(ctx):
    base = dict(CASES["cos_r64_n512_s124"])
    a = _gpu(ctx, _case(**base), "bf16x3g")
    b = _gpu(ctx, _case(**dict(base, div=oracle.DIV_COMPLEX_STEP)), "bf16x3g")
    f = np.isfinite(a)
    assert np.array_equal(f, np.isfinite(b))
    assert np.max(np.abs(a[f] - b[f]) / np.maximum(1.0, np.abs(a[f]))) < 1e-12


@pytest.mark.parametrize("prec", ["bf16x3s", "bf16x3p"])
def test_pull_screened_forms_are_refused(ctx, prec):
    case = _case(**CASES["cos_r64_n512_s124"])
    with pytest.raises(yy.YYError) as e:
        _gpu(ctx, case, prec)
    assert e.value.status == yy.YY_ERR_UNSUPPORTED


def _run(w, dys, prec, form):
    from paper_2509_16896_amd.filter import GpuFilter
    f = GpuFilter(w, prec=prec, form=form)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        torch.cuda.synchronize()
        return f.hist.cpu().numpy()
    finally:
        f.close()


FILTERS = {
    "cubic_r2_n1024_K100_full": (W.cubic_r2(), "fp32", 1e-5),
    "linear_r10_n2048_K10_restart": (W.shrink(W.linear_r10(), n=2048, K=10), "fp32", 1e-5),
    "cubic_r20_n1024_K6_restart_s124": (W.shrink(W.cubic_r100(), r=20, n=1024, K=6), "fp32", 1e-5),
    "cubic_r64_n1024_K6_restart_bf16x3g": (W.shrink(W.cubic_r100(), r=64, n=1024, K=6), "bf16x3g", 1e-3),
    "cubic_r100_n2048_K4_restart_fp32_mfma": (W.shrink(W.cubic_r100(), n=2048, K=4), "fp32_mfma", 1e-5),
}


@pytest.mark.parametrize("name", sorted(FILTERS))
def test_pull_filter_matches_oracle(name):
    w, prec, tol = FILTERS[name]
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys, form=oracle.FORM_PULL)
    got = _run(w, dys, prec, "pull")
    err = float(np.max(np.abs(got - ref["means"])))
    print(f"pull filter {name} [{prec}]: max |mean - oracle| = {err:.3g}; RMSE gpu {W.rmse(got, xs[1:]):.5f} "
          f"oracle {W.rmse(ref['means'], xs[1:]):.5f}", flush=True)
    assert err <= tol


PUSH_VS_PULL = {
    "cubic_r2_n1024": (W.cubic_r2(), "fp32"),
    "linear_r10_n4096": (W.linear_r10(), "fp32"),
    "cubic_r100_n16384": (W.cubic_r100(), "bf16x3g"),
}


@pytest.mark.parametrize("name", sorted(PUSH_VS_PULL))
def test_pull_and_push_filters_track_the_same_path(name):
    w, prec = PUSH_VS_PULL[name]
    xs, dys = W.simulate(w)
    push = _run(w, dys, prec, "push")
    pull = _run(w, dys, prec, "pull")
    rp, rl = W.rmse(push, xs[1:]), W.rmse(pull, xs[1:])
    dm = float(np.max(np.abs(push - pull)))
    print(f"{name} [{prec}]: RMSE push {rp:.5f} pull {rl:.5f}; max |mean(push) - mean(pull)| = {dm:.3g}", flush=True)
    assert np.all(np.isfinite(pull))
    assert abs(rl - rp) <= 0.1 * rp
