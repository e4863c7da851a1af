"""General noise coefficients a = U U^T, b = V V^T, invertible or singular (Sec. 7, Table
tab:generalformulas) on the GPU against the oracle.

The library whitens the node set with W (W^T W = a^+, from its own host eigen-decomposition) and runs
the pairwise kernels unchanged; the oracle forms d^T a^+ d directly with numpy's eigen-decomposition of
a.  Checked: the ranks and log det_+ of the noise object; one prediction in every matrix-core form and
the vector-ALU form, push and pull, against the oracle at 1e-5 on normalised log-densities; the
correction h^T b^+ dy - dt/2 h^T b^+ h; whole filter runs with both coefficients against the oracle's
filter; the batched step refuses such a model.
"""
import math

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


def _coef(r, rank, seed, scale=0.3):
    """U with U U^T = Q diag(lam) Q^T, lam_i in scale * [0.5, 1.5] for i < rank and 0 beyond."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((r, r)))
    lam = np.zeros(r)
    lam[:rank] = scale * (0.5 + rng.random(rank))
    return Q @ np.diag(np.sqrt(lam))


@pytest.mark.parametrize("r,rank", [(3, 3), (8, 6), (64, 64), (100, 97)])
def test_noise_ranks_and_logdet(ctx, r, rank):
    U = _coef(r, rank, r)
    V = _coef(r, max(rank - 1, 1), r + 1)
    nz = yy.yy_noise_create(ctx, r, U, r, V)
    try:
        ra, la, rb, lb = yy.yy_noise_info(nz)
    finally:
        yy.yy_noise_destroy(nz)
    _, lao, rao = oracle.noise_pinv(U)
    _, lbo, rbo = oracle.noise_pinv(V)
    assert (ra, rb) == (rao, rbo)
    assert abs(la - lao) <= 1e-10 * max(1.0, abs(lao)) and abs(lb - lbo) <= 1e-10 * max(1.0, abs(lbo))


CASES = {
    # name: (r, rank of a, n, drift, scales, dt, half)
    "cos_r3_full_n500_s12": (3, 3, 500, oracle.F_COS, (1.0, 2.0), 0.02, 0.6),
    "cos_r8_rank6_n777_s124": (8, 6, 777, oracle.F_COS, (1.0, 2.0, 4.0), 0.02, 0.5),
    "linear_r40_full_n1024_s1": (40, 40, 1024, oracle.F_LINEAR, (1.0,), 0.01, 0.3),
    "cos_r64_rank60_n600_s124": (64, 60, 600, oracle.F_COS, (1.0, 2.0, 4.0), 0.005, 0.3),
    "sinmix_r100_full_n1000_s124": (100, 100, 1000, oracle.F_PAPER_SINMIX, (1.0, 2.0, 4.0), 0.01, 0.3),
}


def _case(ctx, name, form):
    r, rank, n, drift, scales, dt, half = CASES[name]
    U = _coef(r, rank, 7 + r, scale=0.2)
    ap, logdet, k = oracle.noise_pinv(U)
    assert k == rank
    lo, hi = -half * np.ones(r), half * np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, True, r), lo, hi)
    rng = np.random.default_rng(r)
    lw = -3.0 * rng.random(n) - 0.5 * np.sum((x / half) ** 2, axis=1)
    A = W.linear_drift_matrix(r, 0) if drift == oracle.F_LINEAR else None
    om = oracle.OModel(r, r, drift, A, oracle.H_IDENTITY, None, 0.0, 1.0, 1.0)
    c = oracle.kernel_coefficients(scales)
    ref, _ = oracle.propagate_ex(om, scales, c, x, lo, hi, dt, lw, form=form, apinv=ap, logdet_a=logdet)
    return dict(U=U, r=r, n=n, drift=drift, A=A, scales=scales, dt=dt, lo=lo, hi=hi, x=x, lw=lw, ref=ref)


def _gpu(ctx, case, prec, form):
    r, n = case["r"], case["n"]
    nz = yy.yy_noise_create(ctx, r, case["U"], r, None)
    try:
        gm = yy.Model(r, r, case["drift"], case["A"], yy.YY_H_IDENTITY, None, 0.0, 1.0, 1.0, noise=nz)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        yy.yy_propagate(ctx, gm, yy.Scales(case["scales"], form="pull" if form == oracle.FORM_PULL else "push"),
                        prec, n, dev(case["x"].ravel()), next_version(), dev(case["lo"]), dev(case["hi"]),
                        case["dt"], dev(case["lw"]), out)
        return host(out)
    finally:
        yy.yy_noise_destroy(nz)


PREC_PUSH = ["fp32", "fp32_mfma", "bf16x3", "bf16x3g", "bf16x3s", "bf16x3p", "bf16x1"]
PREC_PULL = ["fp32", "fp32_mfma", "bf16x3g"]


@pytest.mark.parametrize("form,prec", [(oracle.FORM_PUSH, p) for p in PREC_PUSH] +
                         [(oracle.FORM_PULL, p) for p in PREC_PULL])
@pytest.mark.parametrize("name", sorted(CASES))
def test_general_noise_propagate_parity(ctx, name, form, prec):
    case = _case(ctx, name, form)
    got = _gpu(ctx, case, prec, form)
    worst, cnt = compare_logw(got, case["ref"], 1e-5)
    print(f"noise {name} form={form} [{prec}]: worst err/allowed = {worst:.3g} over {cnt} nodes", flush=True)
    assert worst <= 1.0
    assert np.array_equal(np.isfinite(got), np.isfinite(case["ref"]))


@pytest.mark.parametrize("r,rank,obs", [(3, 3, "cube"), (8, 5, "cube"), (50, 50, "identity"), (64, 61, "linear")])
def test_general_observation_noise_update(ctx, r, rank, obs):
    rng = np.random.default_rng(3 * r + rank)
    n, dt = 3001, 0.01
    V = _coef(r, rank, 40 + r)
    bp, _, k = oracle.noise_pinv(V)
    assert k == rank
    H = rng.standard_normal((r, r)) / math.sqrt(r) if obs == "linear" else None
    code = {"identity": oracle.H_IDENTITY, "cube": oracle.H_CUBE, "linear": oracle.H_LINEAR}[obs]
    om = oracle.OModel(r, r, oracle.F_ZERO, None, code, H, 0.2, 1.0, 1.0)
    x = rng.standard_normal((n, r)) * 0.7
    dy = rng.standard_normal(r) * 0.1
    lw = rng.standard_normal(n)
    lw[::17] = -np.inf
    ref = oracle.loglik_update_ex(om, x, dy, dt, bp, lw)
    nz = yy.yy_noise_create(ctx, r, None, r, V)
    try:
        gm = yy.Model(r, r, yy.YY_F_ZERO, None, code, H, 0.2, 1.0, 1.0, noise=nz)
        t = dev(lw)
        yy.yy_loglik_update(ctx, gm, n, dev(x.ravel()), dev(dy), dt, t)
        got = host(t)
    finally:
        yy.yy_noise_destroy(nz)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.max(np.abs(got[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin]))) <= 1e-11


def _noisy(w, rank_a, rank_b, seed):
    return W.dataclasses.replace(w, U=_coef(w.r, rank_a, seed, 0.2), V=_coef(w.m, rank_b, seed + 1, 0.2))


FILTERS = {
    "cubic_r6_n2048_K10_full_noise": (_noisy(W.shrink(W.cubic_r100(), r=6, n=2048, K=10), 6, 6, 1), "fp32", 1e-5),
    "cubic_r6_n2048_K10_singular_noise": (_noisy(W.shrink(W.cubic_r100(), r=6, n=2048, K=10), 5, 4, 3), "fp32",
                                          1e-5),
    "cubic_r40_n1024_K6_bf16x3p": (_noisy(W.shrink(W.cubic_r100(), r=40, n=1024, K=6), 40, 38, 5), "bf16x3p", 1e-3),
}


@pytest.mark.parametrize("name", sorted(FILTERS))
def test_general_noise_filter_matches_oracle(name):
    from paper_2509_16896_amd.filter import GpuFilter
    w, prec, tol = FILTERS[name]
    xs, dys = W.simulate(w)
    ap, la, _ = oracle.noise_pinv(w.U)
    bp, _, _ = oracle.noise_pinv(w.V)
    ref = ofilter.run_filter(w, dys, apinv=ap, logdet_a=la, bpinv=bp)
    f = GpuFilter(w, prec=prec)
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
    print(f"noise filter {name} [{prec}]: max |mean - oracle| = {err:.3g}; RMSE gpu {W.rmse(got, xs[1:]):.5f} "
          f"oracle {W.rmse(ref['means'], xs[1:]):.5f}", flush=True)
    assert err <= tol


def test_batch_refuses_general_noise(ctx):
    w = _noisy(W.shrink(W.cubic_r100(), r=8, n=256, K=2), 8, 8, 9)
    nz = yy.yy_noise_create(ctx, 8, w.U, 8, w.V)
    try:
        gm = yy.Model(8, 8, yy.YY_F_COS, None, yy.YY_H_CUBE, None, 0.0, 0.09, 0.09, noise=nz)
        d = torch.zeros(2 * 8, dtype=torch.float64, device="cuda")
        with pytest.raises(yy.YYError) as e:
            yy.yy_batch_create(ctx, [(gm, 256, 0.01, 0.3, 0.3, 2, 2, 1, d)], yy.Scales((1.0,)), "bf16x3g", 0)
        assert e.value.status == yy.YY_ERR_UNSUPPORTED
    finally:
        yy.yy_noise_destroy(nz)
