"""The learned restart proposal on the GPU against the FP64 oracle: forward,
gradients, Adam, sample moments and the learned restart's box decision."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host
from oracle import proposal as OP

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")


@pytest.fixture(scope="module")
def ctx():
    c = yy.yy_create(0, torch.cuda.current_stream())
    yield c
    yy.yy_destroy(c)


def _params(r, H, seed, scale):
    rng = np.random.default_rng(seed)
    p = np.empty(OP.num_params(r, H))
    W1, b1, W2, b2, W3, b3 = OP.unpack(p, r, H)
    W1[...] = rng.uniform(-1, 1, W1.shape) / np.sqrt(r)
    b1[...] = rng.uniform(-0.1, 0.1, b1.shape)
    W2[...] = rng.uniform(-1, 1, W2.shape) / np.sqrt(H)
    b2[...] = rng.uniform(-0.1, 0.1, b2.shape)
    W3[...] = rng.uniform(-scale, scale, W3.shape) / np.sqrt(H)
    b3[...] = rng.uniform(-scale, scale, b3.shape)
    return p.astype(np.float32).astype(np.float64)   # exactly representable in FP32


def _pairs(r, B, seed, R):
    rng = np.random.default_rng(seed)
    xhat = rng.standard_normal((B, r))
    mu = xhat + 0.05 * rng.standard_normal((B, r))
    var = rng.uniform(0.2, 1.5, (B, r)) * (R / OP.KAPPA) ** 2
    return xhat, mu, var


CASES = [(5, 16, 3), (37, 64, 9), (200, 96, 70), (1000, 256, 32)]


@pytest.mark.parametrize("r,H,B", CASES)
def test_forward_and_gradient_parity(ctx, r, H, B):
    R = 0.3
    p = _params(r, H, r, 0.5)
    xhat, mu, var = _pairs(r, B, r + 1, R)
    net = yy.yy_proposal_create(ctx, r, H, 0, dev(p, torch.float32))
    try:
        P = yy.yy_proposal_num_params(net)
        assert P == OP.num_params(r, H)
        out = torch.empty(B * 2 * r, dtype=torch.float32, device="cuda")
        yy.yy_proposal_forward(net, B, dev(xhat), out, r)
        ref_out, _ = OP.forward(p, xhat, r, H)
        got = host(out).reshape(B, 2 * r)
        scale = np.max(np.abs(ref_out))
        assert np.max(np.abs(got - ref_out)) <= 1e-5 * scale
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        grad = torch.empty(P, dtype=torch.float32, device="cuda")
        yy.yy_proposal_train_step(net, B, dev(xhat), dev(mu), dev(var), R, 1e-3, False, loss=loss, grad=grad, r=r)
        ref_loss, ref_g = OP.loss_grad(p, xhat, mu, var, R, r, H)
        assert abs(host(loss)[0] - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
        g = host(grad).astype(np.float64)
        # per parameter block: error <= 1e-4 of the block's largest gradient
        for name, gb, rb in zip(["W1", "b1", "W2", "b2", "W3", "b3"], OP.unpack(g, r, H), OP.unpack(ref_g, r, H)):
            m = np.max(np.abs(rb))
            err = np.max(np.abs(gb - rb))
            assert err <= 1e-4 * m, (name, err, m)
        # parameters are untouched without update
        back = torch.empty(P, dtype=torch.float32, device="cuda")
        yy.yy_proposal_get_params(net, back)
        assert np.array_equal(host(back), p.astype(np.float32))
    finally:
        yy.yy_proposal_destroy(net)


def test_adam_steps_follow_the_oracle(ctx):
    r, H, B, R, lr = 12, 32, 20, 0.4, 2e-3
    p = _params(r, H, 3, 0.3)
    xhat, mu, var = _pairs(r, B, 4, R)
    net = yy.yy_proposal_create(ctx, r, H, 0, dev(p, torch.float32))
    try:
        q, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
        for t in range(1, 6):
            yy.yy_proposal_train_step(net, B, dev(xhat), dev(mu), dev(var), R, lr, True, r=r)
            _, g = OP.loss_grad(q, xhat, mu, var, R, r, H)
            q, m, v = OP.adam_step(q, g, m, v, t, lr)
        got = torch.empty(yy.yy_proposal_num_params(net), dtype=torch.float32, device="cuda")
        yy.yy_proposal_get_params(net, got)
        d = host(got).astype(np.float64) - q
        # Adam's normalised steps move each parameter by about lr per step
        assert np.max(np.abs(d)) <= 0.02 * 5 * lr
        assert np.max(np.abs(q - p)) > 2 * lr
    finally:
        yy.yy_proposal_destroy(net)


def test_default_initialisation_is_the_plain_box(ctx):
    r, H = 20, 64
    net = yy.yy_proposal_create(ctx, r, H, 7, None)
    try:
        xhat = np.random.default_rng(0).standard_normal((3, r))
        out = torch.empty(3 * 2 * r, dtype=torch.float32, device="cuda")
        yy.yy_proposal_forward(net, 3, dev(xhat), out, r)
        assert np.array_equal(host(out), np.zeros(6 * r, np.float32))
        P = yy.yy_proposal_num_params(net)
        prm = torch.empty(P, dtype=torch.float32, device="cuda")
        yy.yy_proposal_get_params(net, prm)
        W1, b1, W2, b2, W3, b3 = OP.unpack(host(prm).astype(np.float64), r, H)
        assert np.all(np.abs(W1) <= 1 / np.sqrt(r)) and np.std(W1) > 0.3 / np.sqrt(r)
        assert np.all(np.abs(W2) <= 1 / np.sqrt(H)) and not np.any(b1) and not np.any(b2)
    finally:
        yy.yy_proposal_destroy(net)


@pytest.mark.parametrize("n,r", [(1000, 3), (5000, 64), (3000, 1000)])
def test_sample_moments(ctx, n, r):
    rng = np.random.default_rng(n + r)
    x = rng.standard_normal((n, r)) * 0.7 + 2.0
    idx = np.sort(rng.integers(0, n, n))
    mean = torch.empty(r, dtype=torch.float64, device="cuda")
    var = torch.empty(r, dtype=torch.float64, device="cuda")
    yy.yy_sample_moments(ctx, n, r, dev(x), dev(idx, torch.int64), mean, var)
    mu, vr = OP.sample_moments(x, idx)
    np.testing.assert_allclose(host(mean), mu, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(host(var), vr, rtol=1e-10, atol=1e-14)


def _restart_case(ctx, r, n, p, H, x_cur, idx, xhat, R, cover_min, ess_min):
    codes = oracle.sobol_codes(r, n, 0, True, 5)
    net = yy.yy_proposal_create(ctx, r, H, 0, dev(p, torch.float32))
    t = {k: torch.empty(v, dtype=torch.float64, device="cuda") for k, v in dict(lo=r, hi=r, x=n * r, lw=n).items()}
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    w = np.full(n, 1.0 / n)
    gidx = dev(idx, torch.int64)
    try:
        yy.yy_get_status(ctx)
        yy.yy_restart(ctx, n, r, dev(codes.view(np.int32).ravel(), torch.int32), dev(x_cur), dev(w), dev(xhat), None,
                      3, R, ess_min, 1, gidx, t["lo"], t["hi"], t["x"], t["lw"], net, cover_min, used)
        flags, _ = yy.yy_get_status(ctx)
    finally:
        yy.yy_proposal_destroy(net)
    ref = OP.learned_restart(p, r, H, x_cur, host(gidx), xhat, R, codes, cover_min, ess_min,
                             oracle.codes_to_points, oracle.is_boundary)
    return codes, t, int(host(used)[0]), flags, ref


@pytest.mark.parametrize("shift,expect_used", [(0.0, True), (5.0, False)])
def test_learned_restart_decision(ctx, shift, expect_used):
    """A network whose output layer predicts a wider box around the samples (used), and one
    that shifts the box far away (coverage fails: the plain box, bit-exact, and the flag)."""
    r, H, n, R = 6, 32, 2048, 0.3
    rng = np.random.default_rng(9)
    p = _params(r, H, 11, 0.0)
    W1, b1, W2, b2, W3, b3 = OP.unpack(p, r, H)
    b3[:r] = shift
    b3[r:] = np.log(2.0)          # half-width 2R
    xhat = rng.standard_normal(r) * 0.5
    x_cur = xhat + rng.standard_normal((n, r)) * (2 * R / OP.KAPPA)
    idx = np.sort(rng.integers(0, n, n))
    codes, t, used, flags, ref = _restart_case(ctx, r, n, p, H, x_cur, idx, xhat, R, 0.9, 8.0)
    ref_used, lo, hi, xn, lw = ref
    assert ref_used == expect_used and used == int(expect_used)
    assert bool(flags & 16) == (not expect_used)
    glo, ghi = host(t["lo"]), host(t["hi"])
    np.testing.assert_allclose(glo, lo, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(ghi, hi, rtol=1e-6, atol=1e-7)
    if not expect_used:
        assert np.array_equal(glo, xhat - R) and np.array_equal(ghi, xhat + R)
    # given the box the GPU chose, the node map and prior are the oracle's exactly
    xo = oracle.codes_to_points(codes, glo, ghi)
    assert np.array_equal(host(t["x"]).reshape(n, r), xo)
    lwo = -0.5 * np.sum((xo - xhat) ** 2, axis=1)
    lwo[oracle.is_boundary(xo, glo, ghi)] = -np.inf
    glw = host(t["lw"])
    assert np.array_equal(np.isinf(glw), np.isinf(lwo))
    f = np.isfinite(lwo)
    np.testing.assert_allclose(glw[f], lwo[f], rtol=1e-13, atol=1e-13)


def test_learned_restart_ess_fallback(ctx):
    """A box so wide that the re-centred prior concentrates on few nodes: the ESS check fails
    after the coverage and log-density checks pass, and the plain nodes are regenerated."""
    r, H, n, R = 4, 16, 512, 0.3
    rng = np.random.default_rng(3)
    p = _params(r, H, 5, 0.0)
    W1, b1, W2, b2, W3, b3 = OP.unpack(p, r, H)
    b3[:r] = 0.0
    b3[r:] = np.log(60.0)          # half-width 18: prior N(x_hat, I) weights a tiny fraction of the nodes
    xhat = np.zeros(r)
    x_cur = rng.standard_normal((n, r)) * 6.0
    idx = np.arange(n)
    codes, t, used, flags, ref = _restart_case(ctx, r, n, p, H, x_cur, idx, xhat, R, 0.5, 200.0)
    ref_used, lo, hi, xn, lw = ref
    assert not ref_used and used == 0 and (flags & 16)
    assert np.array_equal(host(t["lo"]), xhat - R) and np.array_equal(host(t["hi"]), xhat + R)
    assert np.array_equal(host(t["x"]).reshape(n, r), xn)


def test_trained_proposal_gains_over_plain_restart():
    """Cubic sensor r=10 (f = cos, h = x^3, noise std 0.3, n = 4096, dt = 0.01, 100 steps,
    restart every 2 steps with R = 0.3): the network trained on 32 plain-restart runs (their own
    observation paths) lowers the RMSE of the estimate to the true state on 8 held-out paths."""
    import dataclasses

    from paper_2509_16896_amd import proposal as PR
    from paper_2509_16896_amd import workloads as W
    from paper_2509_16896_amd.filter import GpuFilter

    w = W.Workload("cubic_r10_n4096", r=10, n=4096, dt=0.01, K=100, drift=W.F_COS, obs=W.H_CUBE, q=0.09,
                   rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=3.0, restart_every=2, R=0.3, seed=0,
                   precision="fp32")
    X, MU, VAR = PR.collect_pairs(w, range(100, 132))
    assert X.shape == (32 * 48, 10)
    params, losses = PR.train(w, X, MU, VAR, hidden=256, steps=1500, lr=1e-3, log_every=500)
    assert losses[-1][1] < losses[0][1] - 0.3

    def evaluate(prm):
        errs, used, rest = [], 0, 0
        for sd in range(8):
            xs, dys = W.simulate(w, seed=sd)
            f = GpuFilter(w, proposal_params=prm)
            try:
                f.set_observations(dys)
                f.init()
                for k in range(1, w.K + 1):
                    f.step(k)
                est = host(f.hist)
                errs.append(np.sqrt(np.mean((est - xs[1:]) ** 2)))
                used += int(host(f.used_count)[0])
                rest += f.restarts
            finally:
                f.close()
        return float(np.mean(errs)), used / rest

    plain, _ = evaluate(None)
    learned, frac = evaluate(params)
    print(f"plain RMSE {plain:.4f}, learned RMSE {learned:.4f}, learned box used at {frac:.0%} of restarts")
    assert frac >= 0.5
    assert learned <= 0.9 * plain
