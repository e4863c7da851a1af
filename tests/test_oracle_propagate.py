"""Pins of the oracle's prediction step (Sec. 4 kernel operator in push form, Sec. 9 log domain).

Independent references: scipy's multivariate normal log-density for a single
source (drift zero, linear and cosine: pins the Gaussian constant, the
per-scale variance q dt/s, the quadrature weight vol/n, the identity term and
the push orientation of the drift), linearity, shift invariance, conservation
of mass in the resolved regime (sum of coefficients = 1), and the first-order
consistency (L u - u)/dt -> L* u of Theorem thm:1storderkernel.
"""
import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

import oracle
from oracle import F_COS, F_LINEAR, F_ZERO, H_IDENTITY


def _nodes(r, n, half, seed=1):
    lo, hi = -half * np.ones(r), half * np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 1, True, seed), lo, hi)
    return lo, hi, x


def _single_source_expect(x, j0, mean_fn, q, dt, scales, c, lo, hi):
    n, r = x.shape
    logdV = np.sum(np.log(hi - lo)) - np.log(n)
    out = np.empty(n)
    for i in range(n):
        total = 0.0
        for s, cs in zip(scales, c[:-1]):
            tau = dt / s
            total += cs * np.exp(logdV + multivariate_normal.logpdf(x[i], mean_fn(x[j0], tau), q * tau * np.eye(r)))
        if i == j0:
            total += c[-1]
        out[i] = np.log(total) if total > 0 else -np.inf
    return out


@pytest.mark.parametrize("drift", [F_ZERO, F_LINEAR, F_COS])
@pytest.mark.parametrize("scales", [(1.0,), (1.0, 2.0)])
def test_single_source_matches_gaussian_density(oracle_lib, drift, scales):
    r, n, q, dt = 3, 40, 0.7, 0.05
    lo, hi, x = _nodes(r, n, 0.6)
    A = np.array([[-0.5, 0.3, 0.0], [0.1, -0.4, 0.2], [0.0, -0.3, -0.6]])
    model = oracle.OModel(r, r, drift, A if drift == F_LINEAR else None, H_IDENTITY, None, 0.0, q, 1.0)
    if drift == F_ZERO:
        mean_fn = lambda xj, tau: xj
    elif drift == F_LINEAR:
        mean_fn = lambda xj, tau: xj + tau * (A @ xj)
    else:
        mean_fn = lambda xj, tau: xj + tau * np.cos(xj)
    c = oracle.kernel_coefficients(scales)
    j0 = 17
    lw = np.full(n, -np.inf)
    lw[j0] = 0.0
    got, ncl = oracle.propagate(model, scales, c, x, lo, hi, dt, lw)
    expect = _single_source_expect(x, j0, mean_fn, q, dt, scales, c, lo, hi)
    fin = np.isfinite(expect)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.allclose(got[fin], expect[fin], rtol=1e-12, atol=1e-10)
    assert ncl == np.sum(~fin)


def test_linearity_and_shift_invariance(oracle_lib):
    r, n, q, dt = 2, 64, 1.0, 0.05
    lo, hi, x = _nodes(r, n, 1.0)
    model = oracle.OModel(r, r, F_COS, None, H_IDENTITY, None, 0.0, q, 1.0)
    s, c = (1.0,), oracle.kernel_coefficients((1.0,))
    a = np.full(n, -np.inf); a[3] = 0.2
    b = np.full(n, -np.inf); b[40] = -1.1
    ab = np.logaddexp(a, b)
    la, _ = oracle.propagate(model, s, c, x, lo, hi, dt, a)
    lb, _ = oracle.propagate(model, s, c, x, lo, hi, dt, b)
    lab, _ = oracle.propagate(model, s, c, x, lo, hi, dt, ab)
    assert np.allclose(lab, np.logaddexp(la, lb), rtol=1e-13, atol=1e-12)
    lw = -np.random.default_rng(0).random(n) * 4
    l1, _ = oracle.propagate(model, s, c, x, lo, hi, dt, lw)
    l2, _ = oracle.propagate(model, s, c, x, lo, hi, dt, lw + 123.25)
    assert np.allclose(l2 - l1, 123.25, rtol=0, atol=1e-10)


def test_boundary_nodes_are_excluded(oracle_lib):
    r, n = 2, 32
    lo, hi = -np.ones(r), np.ones(r)
    codes = oracle.sobol_codes(r, n, 0, False)  # point 0 has code 0: the corner (-1, -1)
    x = oracle.codes_to_points(codes, lo, hi)
    model = oracle.OModel(r, r, F_ZERO, None, H_IDENTITY, None, 0.0, 1.0, 1.0)
    lw = np.zeros(n)
    out, _ = oracle.propagate(model, (1.0,), (1.0, 0.0), x, lo, hi, 0.1, lw)
    assert out[0] == -np.inf and np.all(np.isfinite(out[1:]))
    lw2 = lw.copy(); lw2[0] = 50.0   # a boundary source contributes nothing
    out2, _ = oracle.propagate(model, (1.0,), (1.0, 0.0), x, lo, hi, 0.1, lw2)
    assert np.array_equal(out, out2)


@pytest.mark.parametrize("scales", [(1.0,), (1.0, 2.0), (1.0, 2.0, 4.0)])
def test_mass_is_conserved_in_the_resolved_regime(oracle_lib, scales):
    # r = 1, 2^11 van der Corput points on [-8, 8] (an equispaced grid), kernel std 0.1 >> spacing
    n, dt = 2048, 0.01
    lo, hi = np.array([-8.0]), np.array([8.0])
    x = oracle.codes_to_points(oracle.sobol_codes(1, n, 0, False), lo, hi)
    model = oracle.OModel(1, 1, F_COS, None, H_IDENTITY, None, 0.0, 1.0, 1.0)
    lw = multivariate_normal.logpdf(x, 0.5, 0.8)
    lw[oracle.is_boundary(x, lo, hi)] = -np.inf
    out, _ = oracle.propagate(model, scales, oracle.kernel_coefficients(scales), x, lo, hi, dt, lw)
    dV = 16.0 / n
    assert abs(dV * np.exp(logsumexp(out)) / (dV * np.exp(logsumexp(lw))) - 1.0) < 1e-9


def test_first_order_consistency(oracle_lib):
    # (L_dt u - u)/dt -> L* u = u''/2 - (f u)'  for u = N(0.3, 0.5^2), f = cos (Theorem thm:1storderkernel)
    n = 4096
    lo, hi = np.array([-5.0]), np.array([5.0])
    x = oracle.codes_to_points(oracle.sobol_codes(1, n, 0, False), lo, hi)[:, 0]
    mu, sd = 0.3, 0.5
    u = np.exp(-0.5 * ((x - mu) / sd) ** 2) / (sd * np.sqrt(2 * np.pi))
    du = -(x - mu) / sd**2 * u
    d2u = ((x - mu) ** 2 / sd**4 - 1 / sd**2) * u
    Lstar = 0.5 * d2u - (-np.sin(x) * u + np.cos(x) * du)
    model = oracle.OModel(1, 1, F_COS, None, H_IDENTITY, None, 0.0, 1.0, 1.0)
    inner = np.abs(x - mu) < 1.5
    errs = []
    for dt in (0.02, 0.01, 0.005):
        out, _ = oracle.propagate(model, (1.0,), (1.0, 0.0), x[:, None], lo, hi, dt, np.log(u))
        errs.append(np.max(np.abs((np.exp(out) - u) / dt - Lstar)[inner]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 0.05 * np.max(np.abs(Lstar[inner]))
    assert np.all(rates > 0.8), (errs, rates)


def test_rows_entry_matches_full(oracle_lib):
    r, n = 3, 100
    lo, hi, x = _nodes(r, n, 0.5)
    model = oracle.OModel(r, r, F_COS, None, H_IDENTITY, None, 0.0, 0.3, 1.0)
    s = (1.0, 2.0, 4.0)
    c = oracle.kernel_coefficients(s)
    lw = -np.random.default_rng(3).random(n)
    full, _ = oracle.propagate(model, s, c, x, lo, hi, 0.02, lw)
    rows = np.array([0, 7, 99, 42])
    part, _ = oracle.propagate_rows(model, s, c, x, lo, hi, 0.02, lw, rows)
    assert np.array_equal(part, full[rows])
