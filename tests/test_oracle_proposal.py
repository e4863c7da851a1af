"""Pins of the oracle's learned restart proposal (CPU only)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import proposal as P


def _params(r, H, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, P.num_params(r, H))


def test_gelu_matches_normal_cdf_and_symmetry():
    x = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(P.gelu(x), x * norm.cdf(x), rtol=1e-14, atol=1e-15)
    # Phi(-x) = 1 - Phi(x)  =>  gelu(-x) = gelu(x) - x
    np.testing.assert_allclose(P.gelu(-x), P.gelu(x) - x, rtol=0, atol=1e-14)
    h = 1e-6
    fd = (P.gelu(x + h) - P.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(P.gelu_grad(x), fd, rtol=1e-8, atol=1e-9)
    assert P.gelu(0.0) == 0.0


def test_loss_is_gaussian_nll_of_samples():
    """The loss written with sample moments equals the mean negative log-density of the
    samples themselves (scipy), up to the dropped constant and the variance floor."""
    rng = np.random.default_rng(1)
    r, T, R = 5, 400, 0.7
    xhat = rng.standard_normal(r)
    out = rng.standard_normal(2 * r) * 0.4
    c, hw = P.learned_box(out, xhat, R)
    s = hw / P.KAPPA
    y = c + rng.standard_normal((T, r)) * 0.5 + 0.2
    mu, var = y.mean(axis=0), y.var(axis=0)
    brute = -norm.logpdf(y, loc=c, scale=s).sum(axis=1).mean()
    floor = P.V0_FRAC * (R / P.KAPPA) ** 2
    loss, _ = P.loss_and_dout(out[None, :], xhat[None, :], mu[None, :], var[None, :] - floor, R)
    assert loss * r + 0.5 * r * math.log(2 * math.pi) == pytest.approx(brute, rel=1e-12)


def test_backward_matches_finite_differences():
    r, H, B, R = 3, 7, 4, 0.5
    rng = np.random.default_rng(2)
    p = _params(r, H, 3)
    xhat = rng.standard_normal((B, r))
    mu = xhat + 0.1 * rng.standard_normal((B, r))
    var = rng.uniform(0.01, 0.2, (B, r))
    _, g = P.loss_grad(p, xhat, mu, var, R, r, H)
    h = 1e-6
    for k in rng.choice(p.size, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (P.loss_grad(pp, xhat, mu, var, R, r, H)[0] - P.loss_grad(pm, xhat, mu, var, R, r, H)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-3), (k, fd, g[k])


def test_adam_first_step_and_convergence():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = P.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected moments equal g and g^2 on the first step
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + P.ADAM_EPS), rtol=1e-13)
    # minimise (p - 3)^2 / 2
    q, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        q, m, v = P.adam_step(q, q - 3.0, m, v, t, 0.05)
    assert abs(q[0] - 3.0) < 1e-3


def test_zero_output_layer_gives_plain_box():
    r, H = 4, 6
    p = _params(r, H, 4)
    W1, b1, W2, b2, W3, b3 = P.unpack(p, r, H)
    W3[...] = 0.0
    b3[...] = 0.0
    xhat = np.array([0.1, -0.2, 0.3, 1.5])
    out, _ = P.forward(p, xhat[None, :], r, H)
    c, hw = P.learned_box(out[0], xhat, 0.3)
    np.testing.assert_array_equal(c, xhat)
    np.testing.assert_allclose(hw, 0.3, rtol=0, atol=0)


def test_training_fits_the_closed_form_optimum():
    """With inputs shared by all pairs only the biases matter at the optimum:
    delta = mean(mu) - x_hat and s^2 = mean(var + floor + (mu - c)^2)."""
    r, H, R = 2, 5, 0.6
    rng = np.random.default_rng(5)
    p = _params(r, H, 6, 0.1)
    xhat = np.tile(np.array([[0.3, -0.4]]), (16, 1))
    mu = xhat + np.array([0.05, -0.02]) + 0.01 * rng.standard_normal((16, r))
    var = np.full((16, r), 0.04)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 4001):
        _, g = P.loss_grad(p, xhat, mu, var, R, r, H)
        p, m, v = P.adam_step(p, g, m, v, t, 3e-3)
    out, _ = P.forward(p, xhat[:1], r, H)
    c, hw = P.learned_box(out[0], xhat[0], R)
    np.testing.assert_allclose(c, mu.mean(axis=0), atol=2e-4)
    floor = P.V0_FRAC * (R / P.KAPPA) ** 2
    s2 = (var + floor + (mu - c) ** 2).mean(axis=0)
    np.testing.assert_allclose(hw / P.KAPPA, np.sqrt(s2), rtol=2e-3)


def test_checks_against_direct_counts():
    rng = np.random.default_rng(7)
    n, r = 200, 3
    x = rng.standard_normal((n, r))
    idx = np.sort(rng.integers(0, n, n))
    c = np.zeros(r)
    half = np.array([1.0, 2.0, 0.5])
    y = x[idx]
    direct = sum(abs(y[t, d] - c[d]) <= half[d] for t in range(n) for d in range(r)) / (n * r)
    assert P.coverage(x, idx, c, half) == pytest.approx(direct, abs=1e-15)
    ld = norm.logpdf(y, loc=c, scale=half / P.KAPPA).sum(axis=1).mean()
    assert P.mean_log_density(x, idx, c, half) == pytest.approx(ld, rel=1e-13)
    mu, var = P.sample_moments(x, idx)
    np.testing.assert_allclose(mu, y.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(var, y.var(axis=0), rtol=1e-12)
    assert P.prior_ess(np.full(50, -3.0)) == pytest.approx(50.0, rel=1e-14)
    lw = np.array([0.0, -np.inf, 0.0, math.log(2.0)])
    assert P.prior_ess(lw) == pytest.approx(16.0 / 6.0, rel=1e-14)
