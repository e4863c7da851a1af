"""Pins of the oracle's correction, normalisation, resampling and restart.

Correction (Sec. 2.2 online stage, Sec. 9 update): for a Gaussian observation
model the Ito-corrected update equals the log-likelihood ratio
log N(dy; h dt, rho2 dt) - log N(dy; 0, rho2 dt) (scipy), and its exponential
has expectation one under dy ~ N(0, rho2 dt) (Remark rem:itocorrection).
Normalisation (Sec. 2.2.2 step 4, Sec. 9): numpy's weighted average and
covariance, scipy's logsumexp, invariance under a constant shift.
Resampling: systematic-resampling count bounds, equal weights give the
identity.  Restart (Sec. 6): containment, box, prior density (scipy).
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import multivariate_normal, norm

import oracle
from oracle import F_ZERO, H_CUBE, H_IDENTITY, H_LINEAR


@pytest.mark.parametrize("obs", [H_IDENTITY, H_CUBE, H_LINEAR])
def test_update_is_gaussian_likelihood_ratio(oracle_lib, obs):
    rng = np.random.default_rng(0)
    n, r, dt, rho2 = 50, 3, 0.01, 0.3
    H = rng.standard_normal((2, r)) if obs == H_LINEAR else None
    m = 2 if obs == H_LINEAR else r
    model = oracle.OModel(r, m, F_ZERO, None, obs, H, 0.4, 1.0, rho2)
    x = rng.standard_normal((n, r))
    dy = rng.standard_normal(m) * 0.1
    lw0 = rng.standard_normal(n)
    lw0[5] = -np.inf
    got = oracle.loglik_update(model, x, dy, dt, lw0)
    h = {H_IDENTITY: x, H_CUBE: (x - 0.4) ** 3}.get(obs, x @ (H.T if H is not None else np.eye(r)))
    sd = math.sqrt(rho2 * dt)
    ratio = np.sum(norm.logpdf(dy[None, :], h * dt, sd) - norm.logpdf(dy[None, :], 0.0, sd), axis=1)
    fin = np.isfinite(lw0)
    assert got[5] == -np.inf
    assert np.allclose(got[fin], lw0[fin] + ratio[fin], rtol=1e-12, atol=1e-10)


def test_ito_correction_makes_the_update_unbiased(oracle_lib):
    rng = np.random.default_rng(1)
    r, dt, rho2 = 4, 0.01, 0.5
    model = oracle.OModel(r, r, F_ZERO, None, H_CUBE, None, 0.0, 1.0, rho2)
    x = np.array([[0.9, -1.1, 0.4, 1.3]])
    draws = 20000
    dys = rng.standard_normal((draws, r)) * math.sqrt(rho2 * dt)
    g = np.array([oracle.loglik_update(model, x, dy, dt, np.zeros(1))[0] for dy in dys])
    vals = np.exp(g)
    assert abs(vals.mean() - 1.0) < 3 * vals.std() / math.sqrt(draws)
    # without the correction the mean is exp(dt |h|^2 / (2 rho2)), visibly above 1
    h2 = np.sum(x**6)
    assert math.exp(0.5 * dt * h2 / rho2) - 1.0 > 6 * vals.std() / math.sqrt(draws)


def test_normalise_matches_numpy(oracle_lib):
    rng = np.random.default_rng(2)
    n, r = 300, 5
    x = rng.standard_normal((n, r))
    lw = rng.standard_normal(n) * 3 + 40.0
    lw[7] = -np.inf
    out = oracle.normalise_moments(x, lw, logZ_acc=1.5)
    w = np.exp(lw - logsumexp(lw))
    assert out["status"] == 0
    assert abs(out["logZ_step"] - logsumexp(lw)) < 1e-12
    assert abs(out["logZ_acc"] - (1.5 + logsumexp(lw))) < 1e-12
    assert np.allclose(out["w"], w, rtol=1e-12, atol=0)
    assert abs(out["w"].sum() - 1.0) < n * 2**-52
    assert np.allclose(out["mean"], np.average(x, axis=0, weights=w), rtol=0, atol=1e-13)
    assert np.allclose(out["cov"], np.cov(x.T, aweights=w, bias=True), rtol=0, atol=1e-13)
    assert abs(out["ess"] - 1.0 / np.sum(w**2)) < 1e-9
    shifted = oracle.normalise_moments(x, lw - 25.0)
    assert np.allclose(shifted["w"], out["w"], rtol=1e-12, atol=0)
    assert np.allclose(shifted["logw"], out["logw"], rtol=0, atol=1e-12)


def test_normalise_reports_all_zero(oracle_lib):
    out = oracle.normalise_moments(np.zeros((4, 2)), np.full(4, -np.inf))
    assert out["status"] == 1 and out["logZ_step"] == -np.inf


def test_resampling_counts_and_order(oracle_lib):
    rng = np.random.default_rng(3)
    n = 997
    w = rng.random(n) ** 4
    w[10:20] = 0.0
    w /= w.sum()
    idx = oracle.resample(w, seed=9, step=4)
    assert np.all(np.diff(idx) >= 0)
    Wi = np.floor(w * 2.0**53).astype(np.int64)
    W = int(Wi.sum())
    counts = np.bincount(idx, minlength=n)
    lo = (n * Wi) // W
    hi = -((-n * Wi) // W)
    assert np.all(counts >= lo) and np.all(counts <= hi)
    assert np.all(counts[10:20] == 0)
    assert not np.array_equal(idx, oracle.resample(w, seed=9, step=5))


def test_equal_weights_resample_to_identity(oracle_lib):
    n = 512
    idx = oracle.resample(np.full(n, 1.0 / n), seed=1, step=1)
    assert np.array_equal(idx, np.arange(n))


def test_restart_box_nodes_and_prior(oracle_lib):
    r, n, R = 4, 256, 0.3
    codes = oracle.sobol_codes(r, n, 0, True, 5)
    mean = np.array([0.5, -1.25, 2.0, 0.0])
    lo, hi, x, lw = oracle.restart_nodes(codes, mean, R)
    assert np.array_equal(lo, mean - R) and np.array_equal(hi, mean + R)
    assert np.all(x >= lo) and np.all(x < hi)
    assert np.array_equal(x, oracle.codes_to_points(codes, lo, hi))
    prior = multivariate_normal.logpdf(x, mean, np.eye(r)) + 0.5 * r * np.log(2 * np.pi)
    fin = np.isfinite(lw)
    assert np.allclose(lw[fin], prior[fin], rtol=0, atol=1e-13)
    assert np.array_equal(~fin, oracle.is_boundary(x, lo, hi))
