"""Parity of every C-ABI call against the FP64 oracle, on identical seeded inputs.

Integer and bit-level results (Sobol codes, node coordinates, resampling
indices, restart nodes) must match exactly; double-precision reductions to
~1e-12; the FP32 pairwise propagation to 1e-5 relative on normalised
log-densities (nodes carrying weight >= 1e-12).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import compare_logw, dev, host, next_version

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")


@pytest.fixture(scope="module")
def ctx():
    c = yy.yy_create(0, torch.cuda.current_stream())
    yield c
    yy.yy_destroy(c)


def _box(r, half=0.6, shift=0.0):
    k = np.arange(r)
    return -half + shift + 0.01 * np.sin(k), half + shift + 0.02 * np.cos(k)


# ---------------------------------------------------------------- Sobol nodes
@pytest.mark.parametrize("r,n,first,scramble", [(1, 1000, 0, False), (2, 1024, 0, False), (7, 1000, 5, True),
                                                (64, 4096, 0, True), (1000, 1536, 3, True), (3, 1, 0, True)])
def test_sobol_bit_exact(ctx, r, n, first, scramble):
    lo, hi = _box(r)
    codes = torch.empty(n * r, dtype=torch.int32, device="cuda")
    x = torch.empty(n * r, dtype=torch.float64, device="cuda")
    yy.yy_nodes_sobol(ctx, r, n, first, scramble, 17, dev(lo), dev(hi), codes, x)
    oc = oracle.sobol_codes(r, n, first, scramble, 17)
    ox = oracle.codes_to_points(oc, lo, hi)
    assert np.array_equal(host(codes).view(np.uint32).reshape(n, r), oc)
    assert np.array_equal(host(x).reshape(n, r), ox)


def test_sobol_codes_only_and_empty(ctx):
    codes = torch.empty(10 * 4, dtype=torch.int32, device="cuda")
    yy.yy_nodes_sobol(ctx, 4, 10, 0, True, 1, None, None, codes, None)
    assert np.array_equal(host(codes).view(np.uint32).reshape(10, 4), oracle.sobol_codes(4, 10, 0, True, 1))
    yy.yy_nodes_sobol(ctx, 4, 0, 0, True, 1, None, None, codes, None)
    with pytest.raises(yy.YYError):
        yy.yy_nodes_sobol(ctx, 4, 10, 2**32 - 5, True, 1, None, None, codes, None)


# ---------------------------------------------------------------- propagation
def _prop_case(r, n, drift, scales, q, dt, half, seed, A=None, scramble=True, lw_kind="random"):
    lo, hi = _box(r, half)
    codes = oracle.sobol_codes(r, n, 0, scramble, seed)
    x = oracle.codes_to_points(codes, lo, hi)
    rng = np.random.default_rng(seed)
    if lw_kind == "random":
        lw = -3.0 * rng.random(n) - 0.5 * np.sum(((x - 0.5 * (lo + hi)) / half) ** 2, axis=1)
    else:
        lw = np.full(n, -np.inf)
        lw[rng.integers(0, n, 3)] = rng.standard_normal(3)
    om = oracle.OModel(r, r, drift, A, oracle.H_IDENTITY, None, 0.0, q, 1.0)
    c = oracle.kernel_coefficients(scales)
    ref, ncl = oracle.propagate(om, scales, c, x, lo, hi, dt, lw)
    gm = yy.Model(r, r, drift, A, yy.YY_H_IDENTITY, None, 0.0, q, 1.0)
    return dict(lo=lo, hi=hi, x=x, lw=lw, ref=ref, ncl=ncl, gm=gm, scales=scales, dt=dt, n=n, r=r)


def _gpu_prop(ctx, case, prec):
    n = case["n"]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    xd = dev(case["x"].ravel())
    yy.yy_propagate(ctx, case["gm"], yy.Scales(case["scales"]), prec, n, xd, next_version(), dev(case["lo"]),
                    dev(case["hi"]), case["dt"], dev(case["lw"]), out)
    return host(out)


PROP_CASES = {
    # the plain cubic-sensor shape: r=2, unit noise, n=1024 on a box, scales {1,2}
    "cubic_r2_n1024_s12": dict(r=2, n=1024, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.01, half=4.0, seed=0),
    "cubic_r2_ragged_n1000": dict(r=2, n=1000, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.01, half=4.0, seed=1),
    "linear_r10_n4096": dict(r=10, n=4096, drift=oracle.F_LINEAR, scales=(1.0,), q=0.1, dt=0.01, half=0.75, seed=2),
    "cos_r5_n777_s124": dict(r=5, n=777, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.3, dt=0.05, half=0.8, seed=3),
    "cos_r17_n300_s1": dict(r=17, n=300, drift=oracle.F_COS, scales=(1.0,), q=0.5, dt=0.02, half=1.0, seed=4),
    "zero_r3_n65_sparse": dict(r=3, n=65, drift=oracle.F_ZERO, scales=(1.0, 2.0), q=1.0, dt=0.05, half=1.0, seed=5,
                               lw_kind="sparse"),
    "cos_r2_unscrambled_boundary": dict(r=2, n=256, drift=oracle.F_COS, scales=(1.0,), q=1.0, dt=0.02, half=2.0,
                                        seed=6, scramble=False),
    # the paper's large-scale drift (bidiagonal sin mix), its r=10 size and unit noise
    "sinmix_r10_n100_s124": dict(r=10, n=100, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0, dt=0.01,
                                 half=0.3, seed=7),
}


@pytest.mark.parametrize("name", sorted(PROP_CASES))
def test_propagate_fp32_parity(ctx, name):
    kw = dict(PROP_CASES[name])
    A = None
    if kw["drift"] == oracle.F_LINEAR:
        from paper_2509_16896_amd.workloads import linear_drift_matrix
        A = linear_drift_matrix(kw["r"], 0)
    case = _prop_case(A=A, **kw)
    got = _gpu_prop(ctx, case, "fp32")
    worst, cnt = compare_logw(got, case["ref"], 1e-5)
    print(f"{name}: worst err/allowed = {worst:.3g} over {cnt} nodes")
    assert worst <= 1.0
    # boundary targets are -inf on both sides
    bnd = oracle.is_boundary(case["x"], case["lo"], case["hi"])
    assert np.all(np.isneginf(got[bnd]))


def test_propagate_is_deterministic(ctx):
    case = _prop_case(5, 777, oracle.F_COS, (1.0, 2.0, 4.0), 0.3, 0.05, 0.8, 3)
    a = _gpu_prop(ctx, case, "fp32")
    b = _gpu_prop(ctx, case, "fp32")
    assert np.array_equal(a, b)


def test_propagate_rejects_bad_arguments(ctx):
    case = _prop_case(2, 64, oracle.F_COS, (1.0,), 1.0, 0.01, 1.0, 0)
    lw = dev(case["lw"])
    with pytest.raises(yy.YYError):
        yy.yy_propagate(ctx, case["gm"], yy.Scales((1.0,)), "fp32", 64, dev(case["x"].ravel()), 1,
                        dev(case["lo"]), dev(case["hi"]), 0.01, lw, lw)   # aliasing in/out
    with pytest.raises(yy.YYError):
        yy.yy_propagate(ctx, case["gm"], yy.Scales((1.0,)), "fp32", 64, dev(case["x"].ravel()), 1,
                        dev(case["lo"]), dev(case["hi"]), -0.01, lw, torch.empty_like(lw))


# ---------------------------------------------------------------- correction / normalisation
@pytest.mark.parametrize("obs", ["identity", "cube", "linear"])
def test_loglik_parity(ctx, obs):
    rng = np.random.default_rng(7)
    n, r, dt, rho2 = 1000, 33, 0.005, 0.09
    H = rng.standard_normal((5, r)) if obs == "linear" else None
    m = 5 if obs == "linear" else r
    code = {"identity": 0, "cube": 1, "linear": 2}[obs]
    x = rng.standard_normal((n, r)) * 0.4 + 1.0
    dy = rng.standard_normal(m) * 0.05
    lw = rng.standard_normal(n)
    lw[[3, 500]] = -np.inf
    ref = oracle.loglik_update(oracle.OModel(r, m, 0, None, code, H, 0.1, 1.0, rho2), x, dy, dt, lw)
    g = dev(lw)
    yy.yy_loglik_update(ctx, yy.Model(r, m, 0, None, code, H, 0.1, 1.0, rho2), n, dev(x.ravel()), dev(dy), dt, g)
    got = host(g)
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    f = np.isfinite(ref)
    assert np.allclose(got[f], ref[f], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("n,r", [(1, 1), (300, 5), (70001, 3), (2048, 300)])
def test_normalise_parity(ctx, n, r):
    rng = np.random.default_rng(n + r)
    x = rng.standard_normal((n, r))
    lw = rng.standard_normal(n) * 4 + 100.0
    if n > 10:
        lw[::7] = -np.inf
    ref = oracle.normalise_moments(x, lw, logZ_acc=2.0)
    d = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in
         dict(w=n, lz=1, acc=1, mean=r, cov=r * r, ess=1).items()}
    d["acc"].fill_(2.0)
    g = dev(lw)
    yy.yy_normalise_moments(ctx, n, r, dev(x.ravel()), g, d["w"], d["lz"], d["acc"], d["mean"], d["cov"], d["ess"])
    assert np.allclose(host(g)[np.isfinite(lw)], ref["logw"][np.isfinite(lw)], rtol=0, atol=1e-12)
    assert np.allclose(host(d["w"]), ref["w"], rtol=1e-12, atol=1e-300)
    assert abs(host(d["lz"])[0] - ref["logZ_step"]) < 1e-12
    assert abs(host(d["acc"])[0] - ref["logZ_acc"]) < 1e-12
    assert np.allclose(host(d["mean"]), ref["mean"], rtol=0, atol=1e-13)
    assert np.allclose(host(d["cov"]).reshape(r, r), ref["cov"], rtol=0, atol=1e-13)
    assert abs(host(d["ess"])[0] - ref["ess"]) <= 1e-11 * ref["ess"]


@pytest.mark.parametrize("n,r", [(300, 5), (70001, 3)])
def test_normalise_without_moments(ctx, n, r):
    """mean = NULL: the log-weights, logZ and ESS of the full call, x never read."""
    rng = np.random.default_rng(n + 3 * r)
    x = rng.standard_normal((n, r))
    lw = rng.standard_normal(n) * 4 - 20.0
    lw[::5] = -np.inf
    ref = oracle.normalise_moments(x, lw, logZ_acc=1.5)
    d = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in dict(lz=1, acc=1, ess=1).items()}
    d["acc"].fill_(1.5)
    g = dev(lw)
    nan_x = torch.full((n * r,), float("nan"), dtype=torch.float64, device="cuda")   # would poison a mean
    yy.yy_normalise_moments(ctx, n, r, nan_x, g, None, d["lz"], d["acc"], None, None, d["ess"])
    f = np.isfinite(lw)
    assert np.array_equal(np.isfinite(host(g)), f)
    assert np.allclose(host(g)[f], ref["logw"][f], rtol=0, atol=1e-12)
    assert abs(host(d["lz"])[0] - ref["logZ_step"]) < 1e-12
    assert abs(host(d["acc"])[0] - ref["logZ_acc"]) < 1e-12
    assert abs(host(d["ess"])[0] - ref["ess"]) <= 1e-11 * ref["ess"]
    with pytest.raises(yy.YYError):
        cov = torch.zeros(r * r, dtype=torch.float64, device="cuda")
        yy.yy_normalise_moments(ctx, n, r, nan_x, g, None, d["lz"], d["acc"], None, cov, d["ess"])


def test_normalise_flags_all_zero(ctx):
    n, r = 100, 2
    d = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in dict(lz=1, acc=1, mean=r, ess=1).items()}
    yy.yy_get_status(ctx)
    g = dev(np.full(n, -np.inf))
    yy.yy_normalise_moments(ctx, n, r, dev(np.zeros(n * r)), g, None, d["lz"], d["acc"], d["mean"], None, d["ess"])
    flags, _ = yy.yy_get_status(ctx)
    assert flags & yy.YY_FLAG_ALL_ZERO
    assert host(d["lz"])[0] == -np.inf and host(d["acc"])[0] == 0.0


@pytest.mark.parametrize("n,r,obs", [(1, 2, "cube"), (777, 64, "identity"), (3000, 300, "cube"),
                                     (5001, 1000, "cube"), (700, 33, "cube"), (300, 2048, "identity")])
def test_loglik_normalise_one_call(ctx, n, r, obs):
    """yy_loglik_normalise against yy_loglik_update + yy_normalise_moments and against the oracle's
    two steps (one pass over x for even r up to 1024; the two calls for r = 33 and r = 2048)."""
    rng = np.random.default_rng(n + r)
    code = {"identity": 0, "cube": 1}[obs]
    x = rng.standard_normal((n, r)) * 0.4 + 0.2
    dy = rng.standard_normal(r) * 0.05
    lw = rng.standard_normal(n) * 3 - 10.0
    if n > 10:
        lw[::9] = -np.inf
    dt, rho2 = 0.005, 0.09
    gm = yy.Model(r, r, 0, None, code, None, 0.1, 1.0, rho2)
    xd, dyd = dev(x.ravel()), dev(dy)

    def run(one):
        d = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in
             dict(w=n, lz=1, acc=1, mean=r, ess=1).items()}
        d["acc"].fill_(0.5)
        g = dev(lw)
        if one:
            yy.yy_loglik_normalise(ctx, gm, n, xd, dyd, dt, g, d["w"], d["lz"], d["acc"], d["mean"], d["ess"])
        else:
            yy.yy_loglik_update(ctx, gm, n, xd, dyd, dt, g)
            yy.yy_normalise_moments(ctx, n, r, xd, g, d["w"], d["lz"], d["acc"], d["mean"], None, d["ess"])
        out = {k: host(v) for k, v in d.items()}
        out["logw"] = host(g)
        return out

    a, b = run(True), run(False)
    om = oracle.OModel(r, r, 0, None, code, None, 0.1, 1.0, rho2)
    o = oracle.normalise_moments(x, oracle.loglik_update(om, x, dy, dt, lw), logZ_acc=0.5, want_cov=False)
    ref = dict(w=o["w"], lz=[o["logZ_step"]], acc=[o["logZ_acc"]], mean=o["mean"], ess=[o["ess"]], logw=o["logw"])
    f = np.isfinite(lw)
    for other in (b, ref):
        assert np.array_equal(np.isfinite(a["logw"]), f)
        assert np.allclose(a["logw"][f], np.asarray(other["logw"])[f], rtol=0, atol=1e-12)
        assert np.allclose(a["w"], other["w"], rtol=1e-11, atol=1e-300)
        assert abs(a["lz"][0] - other["lz"][0]) < 1e-12
        assert abs(a["acc"][0] - other["acc"][0]) < 1e-12
        assert np.allclose(a["mean"], other["mean"], rtol=0, atol=1e-13)
        assert abs(a["ess"][0] - other["ess"][0]) <= 1e-11 * other["ess"][0]
    yy.yy_get_status(ctx)


def test_loglik_normalise_all_zero(ctx):
    n, r = 100, 4
    gm = yy.Model(r, r, 0, None, 1, None, 0.0, 1.0, 0.09)
    d = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in dict(lz=1, acc=1, mean=r, ess=1).items()}
    d["mean"].fill_(7.0)
    yy.yy_get_status(ctx)
    g = dev(np.full(n, -np.inf))
    yy.yy_loglik_normalise(ctx, gm, n, dev(np.zeros(n * r)), dev(np.zeros(r)), 0.01, g, None, d["lz"], d["acc"],
                           d["mean"], d["ess"])
    flags, _ = yy.yy_get_status(ctx)
    assert flags & yy.YY_FLAG_ALL_ZERO
    assert host(d["lz"])[0] == -np.inf and host(d["acc"])[0] == 0.0
    assert np.all(host(d["mean"]) == 7.0) and np.all(host(g) == -np.inf)


# ---------------------------------------------------------------- resampling / restart
@pytest.mark.parametrize("n", [1, 255, 256, 4099, 65536])
def test_resample_bit_exact(ctx, n):
    rng = np.random.default_rng(n)
    w = rng.random(n) ** 6
    w[: n // 10] = 0.0
    w /= w.sum()
    ref = oracle.resample(w, seed=77, step=12)
    r = 2
    idx = torch.empty(n, dtype=torch.int64, device="cuda")
    codes = torch.zeros(n * r, dtype=torch.int32, device="cuda")
    tmp = {k: torch.empty(v, dtype=torch.float64, device="cuda") for k, v in dict(lo=r, hi=r, x=n * r, lw=n).items()}
    yy.yy_restart(ctx, n, r, codes, None, dev(w), dev(np.zeros(r)), None, 12, 0.3, 0.0, 77, idx, tmp["lo"], tmp["hi"],
                  tmp["x"], tmp["lw"])
    assert np.array_equal(host(idx), ref)


@pytest.mark.parametrize("r,n", [(3, 500), (1000, 2048)])
def test_restart_nodes_bit_exact(ctx, r, n):
    codes = oracle.sobol_codes(r, n, 0, True, 4)
    mean = np.random.default_rng(r).standard_normal(r)
    lo, hi, x, lw = oracle.restart_nodes(codes, mean, 0.3)
    t = {k: torch.empty(v, dtype=torch.float64, device="cuda") for k, v in dict(lo=r, hi=r, x=n * r, lw=n).items()}
    yy.yy_restart(ctx, n, r, dev(codes.view(np.int32).ravel(), torch.int32), None, None, dev(mean), None, 1, 0.3, 0.0, 0,
                  None, t["lo"], t["hi"], t["x"], t["lw"])
    assert np.array_equal(host(t["lo"]), lo) and np.array_equal(host(t["hi"]), hi)
    assert np.array_equal(host(t["x"]).reshape(n, r), x)
    glw = host(t["lw"])
    assert np.array_equal(np.isinf(glw), np.isinf(lw))
    f = np.isfinite(lw)
    assert np.allclose(glw[f], lw[f], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- matrix-core propagation
MFMA_CASES = {
    # r >= 32: the distance expansion runs on the matrix cores, near pairs exactly
    "sinmix_r50_n300_s124": dict(r=50, n=300, drift=oracle.F_PAPER_SINMIX, scales=(1.0, 2.0, 4.0), q=1.0, dt=0.01,
                                 half=0.3, seed=13),
    "cos_r64_n512_s124": dict(r=64, n=512, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09, dt=0.005, half=0.3,
                              seed=11),
    "cos_r100_n1000_ragged_s124": dict(r=100, n=1000, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09, dt=0.005,
                                       half=0.3, seed=12),
    "cos_r33_n300_s1": dict(r=33, n=300, drift=oracle.F_COS, scales=(1.0,), q=0.5, dt=0.02, half=0.5, seed=13),
    "linear_r128_n2048_s12": dict(r=128, n=2048, drift=oracle.F_LINEAR, scales=(1.0, 2.0), q=0.1, dt=0.01, half=0.4,
                                  seed=14),
    # many near pairs (wide kernel, small box): exercises the exact near-pair path heavily
    "cos_r40_n1024_dense_near": dict(r=40, n=1024, drift=oracle.F_COS, scales=(1.0,), q=2.0, dt=0.05, half=0.25,
                                     seed=15),
    "cos_r36_n2048_near_s12": dict(r=36, n=2048, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.06, half=0.4,
                                   seed=18),
    "zero_r48_n257_sparse": dict(r=48, n=257, drift=oracle.F_ZERO, scales=(1.0, 2.0), q=1.0, dt=0.05, half=0.5,
                                 seed=16, lw_kind="sparse"),
    "cos_r64_n512_unscrambled_boundary": dict(r=64, n=512, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.09,
                                              dt=0.005, half=0.3, seed=17, scramble=False),
    # edges: r = 1 (K padded from 1), r at the K padding boundaries, the largest r, four scales, two nodes
    "cos_r1_n300_s12_dense": dict(r=1, n=300, drift=oracle.F_COS, scales=(1.0, 2.0), q=1.0, dt=0.02, half=2.0,
                                  seed=19),
    "cos_r31_n400_s124": dict(r=31, n=400, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0), q=0.3, dt=0.02, half=0.5,
                              seed=20),
    "cos_r65_n300_s1248": dict(r=65, n=300, drift=oracle.F_COS, scales=(1.0, 2.0, 4.0, 8.0), q=0.2, dt=0.02,
                               half=0.4, seed=21),
    "cos_r3600_n160_s12_max_r": dict(r=3600, n=160, drift=oracle.F_COS, scales=(1.0, 2.0), q=0.09, dt=0.005,
                                     half=0.05, seed=22),
    "zero_r96_n2_s1": dict(r=96, n=2, drift=oracle.F_ZERO, scales=(1.0,), q=1.0, dt=0.05, half=0.5, seed=23),
}


@pytest.mark.parametrize("prec", ["fp32_mfma", "bf16x3", "bf16x3g", "bf16x3s", "bf16x3p", "bf16x1"])
@pytest.mark.parametrize("name", sorted(MFMA_CASES))
def test_propagate_mfma_parity(ctx, name, prec):
    kw = dict(MFMA_CASES[name])
    A = None
    if kw["drift"] == oracle.F_LINEAR:
        from paper_2509_16896_amd.workloads import linear_drift_matrix
        A = linear_drift_matrix(kw["r"], 0)
    case = _prop_case(A=A, **kw)
    got = _gpu_prop(ctx, case, prec)
    worst, cnt = compare_logw(got, case["ref"], 1e-5)
    print(f"{name} [{prec}]: worst err/allowed = {worst:.3g} over {cnt} nodes")
    assert worst <= 1.0
    bnd = oracle.is_boundary(case["x"], case["lo"], case["hi"])
    assert np.all(np.isneginf(got[bnd]))
    # the matrix-core forms reproduce the plain FP32 form up to summation order
    plain = _gpu_prop(ctx, case, "fp32")
    f = np.isfinite(plain)
    assert np.array_equal(np.isfinite(got), f)
    assert np.max(np.abs(got[f] - plain[f]) / np.maximum(1.0, np.abs(plain[f]))) < 2e-6


@pytest.mark.parametrize("prec", ["fp32", "fp32_mfma", "bf16x3", "bf16x3g", "bf16x3s", "bf16x3p", "bf16x1"])
def test_propagate_single_node_raw_value(ctx, prec):
    """One node: the only source is the target itself, so the raw (unnormalised) value is
    the signed combination of the self-pair Gaussian densities -- constants included."""
    for r in (1, 40, 200):
        case = _prop_case(r, 1, oracle.F_COS, (1.0, 2.0, 4.0), 0.09, 0.005, 0.3, 30 + r)
        got = _gpu_prop(ctx, case, prec)
        ref = case["ref"]
        assert np.isfinite(ref[0]) == np.isfinite(got[0])
        if np.isfinite(ref[0]):
            assert abs(got[0] - ref[0]) <= 1e-5 * max(1.0, abs(ref[0])), (r, got[0], ref[0])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3g", "bf16x3s", "bf16x3p"])
def test_propagate_empty_input(ctx, prec):
    gm = yy.Model(8, 8, yy.YY_F_COS, None, yy.YY_H_IDENTITY, None, 0.0, 0.1, 1.0)
    z = torch.zeros(8, dtype=torch.float64, device="cuda")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    yy.yy_propagate(ctx, gm, yy.Scales((1.0,)), prec, 0, e, next_version(), z, z + 1.0, 0.01, e, e)

