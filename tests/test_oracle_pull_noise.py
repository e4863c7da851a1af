"""Pins of the oracle's pull-form kernel (Sec. 4.1, Theorem thm:1storderkernel, eq. kernel), its divergence
(closed forms and the complex-step sum of Sec. 8) and the general noise coefficients a = U U^T, b = V V^T
with the pseudo-inverse of the singular case (Sec. 7, Table tab:generalformulas).

* Divergence: closed form and complex step against mpmath's numerical derivative at 30 digits.
* Pull form: single-source values against scipy's Gaussian log-density centred at x_i - tau f(x_i) times
  exp(-tau div f(x_i)); 50-digit linear-domain double sums for n <= 64 with one to three signed scales;
  first-order consistency with one scale and second order with {1, 2, 4}; agreement with the push form
  to the same orders.
* General noise: a = q I reproduces the isotropic oracle; single sources against scipy's full-covariance
  Gaussian (invertible a) and against scipy in the coordinates of a's range (singular a, where the table
  keeps the constant (2 pi dt)^{-r/2} det_+(a)^{-1/2}); the observation update against scipy's likelihood
  ratio with covariance b dt (invertible b) and in b's range coordinates (singular b), and its invariance
  under components in b's null space.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
from oracle import (DIV_CLOSED, DIV_COMPLEX_STEP, F_COS, F_LINEAR, F_PAPER_SINMIX, F_ZERO, FORM_PULL, FORM_PUSH,
                    H_CUBE, H_IDENTITY)


def _model(r, drift, A=None, q=1.0, obs=H_IDENTITY, rho2=1.0):
    return oracle.OModel(r, r, drift, A if drift == F_LINEAR else None, obs, None, 0.0, q, rho2)


def _f_mp(drift, A, z, k):
    """f_k at the mpmath point z (a list)."""
    r = len(z)
    if drift == F_ZERO:
        return mpmath.mpf(0)
    if drift == F_COS:
        return mpmath.cos(z[k])
    if drift == F_PAPER_SINMIX:
        nxt = z[k + 1] if k + 1 < r else 0
        return mpmath.sin(z[k]) * (-0.5 * z[k] + 0.1 * nxt) + mpmath.sin(2 * z[k]) * (-0.3 * z[k] + 0.3 * nxt)
    return mpmath.fsum(mpmath.mpf(A[k, l]) * z[l] for l in range(r))


@pytest.mark.parametrize("drift", [F_ZERO, F_COS, F_LINEAR, F_PAPER_SINMIX])
@pytest.mark.parametrize("r", [1, 5])
def test_divergence_closed_form_and_complex_step_against_numerical_derivative(oracle_lib, drift, r):
    rng = np.random.default_rng(10 * r + drift)
    A = rng.standard_normal((r, r))
    m = _model(r, drift, A)
    x = rng.standard_normal((6, r)) * 1.5
    closed = oracle.divergence(m, x, DIV_CLOSED)
    cstep = oracle.divergence(m, x, DIV_COMPLEX_STEP, 1e-20)
    with mpmath.workdps(30):
        for i in range(x.shape[0]):
            ref = mpmath.mpf(0)
            for k in range(r):
                def fk(t, k=k):
                    z = [mpmath.mpf(float(v)) for v in x[i]]
                    z[k] = t
                    return _f_mp(drift, A, z, k)
                ref += mpmath.diff(fk, mpmath.mpf(float(x[i, k])))
            tol = 1e-13 * max(1.0, abs(float(ref)))
            assert abs(closed[i] - float(ref)) <= tol, (i, closed[i], ref)
            assert abs(cstep[i] - float(ref)) <= tol, (i, cstep[i], ref)


def _nodes(r, n, half, seed=1, first=1):
    lo, hi = -half * np.ones(r), half * np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, first, True, seed), lo, hi)
    return lo, hi, x


@pytest.mark.parametrize("drift", [F_ZERO, F_LINEAR, F_COS, F_PAPER_SINMIX])
@pytest.mark.parametrize("scales", [(1.0,), (1.0, 2.0)])
@pytest.mark.parametrize("div_mode", [DIV_CLOSED, DIV_COMPLEX_STEP])
def test_pull_single_source_matches_gaussian_density(oracle_lib, drift, scales, div_mode):
    r, n, q, dt = 3, 40, 0.7, 0.05
    lo, hi, x = _nodes(r, n, 0.6)
    A = np.array([[-0.5, 0.3, 0.0], [0.1, -0.4, 0.2], [0.0, -0.3, -0.6]])
    m = _model(r, drift, A, q)
    F = oracle.drift(m, x)
    div = oracle.divergence(m, x, DIV_CLOSED)
    c = oracle.kernel_coefficients(scales)
    j0 = 17
    lw = np.full(n, -np.inf)
    lw[j0] = 0.0
    got, ncl = oracle.propagate_ex(m, scales, c, x, lo, hi, dt, lw, form=FORM_PULL, div_mode=div_mode)
    logdV = np.sum(np.log(hi - lo)) - np.log(n)
    expect = np.empty(n)
    for i in range(n):
        total = 0.0
        for s, cs in zip(scales, c[:-1]):
            tau = dt / s
            dens = multivariate_normal.logpdf(x[j0], x[i] - tau * F[i], q * tau * np.eye(r)) - tau * div[i]
            total += cs * np.exp(logdV + dens)
        if i == j0:
            total += c[-1]
        expect[i] = np.log(total) if total > 0 else -np.inf
    fin = np.isfinite(expect)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.allclose(got[fin], expect[fin], rtol=1e-12, atol=1e-10)
    assert ncl == np.sum(~fin)


def _coefficients(S):
    with mpmath.workdps(50):
        r2 = mpmath.sqrt(2)
        return {1: ((1.0,), [mpmath.mpf(1), mpmath.mpf(0)]),
                2: ((1.0, 2.0), [-r2 - 1, 4 + 2 * r2, -2 - r2]),
                3: ((1.0, 2.0, 4.0), [1 + r2, -8 - 6 * r2, 16 + 8 * r2, -8 - 3 * r2])}[S]


@pytest.mark.parametrize("S", [1, 2, 3])
@pytest.mark.parametrize("drift", [F_COS, F_LINEAR])
@pytest.mark.parametrize("r", [1, 3])
def test_pull_prediction_equals_50_digit_double_sum(oracle_lib, r, drift, S):
    n, q, dt = 48, 0.8, 0.07
    lo, hi = -np.ones(r), np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, False), lo, hi)   # point 0: a boundary corner
    rng = np.random.default_rng(7 * r + S + drift)
    lw = -3.0 * rng.random(n)
    lw[[3, 9]] = -np.inf
    lw[0] = 2.0
    lw[n // 2] = 4.0
    A = rng.standard_normal((r, r)) * 0.5 - np.eye(r)
    m = _model(r, drift, A, q)
    scales, c_mp = _coefficients(S)
    c = np.array([float(v) for v in c_mp])
    got, nclamped = oracle.propagate_ex(m, scales, c, x, lo, hi, dt, lw, form=FORM_PULL)
    nref = 0
    with mpmath.workdps(50):
        X = [[mpmath.mpf(float(v)) for v in row] for row in x]
        bnd = [any(abs(x[i, k] - lo[k]) <= 1e-12 or abs(hi[k] - x[i, k]) <= 1e-12 for k in range(r)) for i in range(n)]
        dV = mpmath.fprod(mpmath.mpf(float(hi[k] - lo[k])) for k in range(r)) / n
        E = [mpmath.e ** mpmath.mpf(float(v)) if np.isfinite(v) else mpmath.mpf(0) for v in lw]
        for i in range(n):
            if bnd[i]:
                assert got[i] == -np.inf
                continue
            Fi = [_f_mp(drift, A, X[i], k) for k in range(r)]
            divi = mpmath.fsum(mpmath.diff(lambda t, k=k: _f_mp(drift, A, X[i][:k] + [t] + X[i][k + 1:], k), X[i][k])
                               for k in range(r))
            total, absum = mpmath.mpf(0), mpmath.mpf(0)
            for s, cs in zip(scales, c_mp[:-1]):
                tau = mpmath.mpf(dt) / s
                sd = mpmath.sqrt(mpmath.mpf(q) * tau)
                acc = mpmath.mpf(0)
                for j in range(n):
                    if bnd[j] or E[j] == 0:
                        continue
                    acc += mpmath.fprod(mpmath.npdf(X[j][k], X[i][k] - tau * Fi[k], sd) for k in range(r)) * E[j]
                term = dV * acc * mpmath.e ** (-tau * divi)
                total += cs * term
                absum += abs(cs) * term
            total += c_mp[-1] * E[i]
            absum += abs(c_mp[-1]) * E[i]
            if total <= 0:
                nref += absum > 0
                assert got[i] == -np.inf, (i, got[i])
                continue
            val = float(mpmath.log(total))
            assert abs(got[i] - val) <= 1e-13 * max(1.0, abs(val)) + 4e-16 * float(absum / total), (i, got[i], val)
    assert nclamped == nref


def test_pull_form_consistency_orders_and_agreement_with_push(oracle_lib):
    """(L u - u)/dt - L* u: first order with one scale, second with {1,2,4}; the pull and push forms agree
    to the same orders (Theorem thm:1storderkernel, Sec. 4.3.3)."""
    n = 4096
    lo, hi = np.array([-5.0]), np.array([5.0])
    x = oracle.codes_to_points(oracle.sobol_codes(1, n, 0, False), lo, hi)[:, 0]
    mu, sd = 0.3, 0.5
    u = np.exp(-0.5 * ((x - mu) / sd) ** 2) / (sd * np.sqrt(2 * np.pi))
    du = -(x - mu) / sd**2 * u
    d2u = ((x - mu) ** 2 / sd**4 - 1 / sd**2) * u
    Lstar = 0.5 * d2u - (-np.sin(x) * u + np.cos(x) * du)
    m = _model(1, F_COS)
    inner = np.abs(x - mu) < 1.5
    for scales, lo_rate, hi_rate in (((1.0,), 0.85, 1.2), ((1.0, 2.0, 4.0), 1.75, 2.3)):
        c = oracle.kernel_coefficients(scales)
        errs, diffs = [], []
        for dt in (0.04, 0.02, 0.01):
            pull, _ = oracle.propagate_ex(m, scales, c, x[:, None], lo, hi, dt, np.log(u), form=FORM_PULL)
            push, _ = oracle.propagate_ex(m, scales, c, x[:, None], lo, hi, dt, np.log(u), form=FORM_PUSH)
            errs.append(np.max(np.abs((np.exp(pull) - u) / dt - Lstar)[inner]))
            diffs.append(np.max(np.abs((np.exp(pull) - np.exp(push)) / dt)[inner]))
        rate = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        rdiff = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
        assert np.all(rate > lo_rate) and np.all(rate < hi_rate), (scales, errs, rate)
        assert np.all(rdiff > lo_rate - 0.15), (scales, diffs, rdiff)


# ---------------------------------------------------------------------------------------------------
# general noise coefficients (Sec. 7)

def _random_U(r, rank, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((r, r)))
    lam = np.zeros(r)
    lam[:rank] = 0.2 + rng.random(rank)
    return Q @ np.diag(np.sqrt(lam)), Q, lam


def test_noise_pinv_moore_penrose_and_log_pseudo_determinant(oracle_lib):
    U, Q, lam = _random_U(6, 4, 1)
    ap, logdet, rank = oracle.noise_pinv(U)
    assert rank == 4
    assert abs(logdet - np.sum(np.log(lam[:4]))) < 1e-12
    a = U @ U.T
    # Moore-Penrose conditions
    assert np.allclose(a @ ap @ a, a, atol=1e-12) and np.allclose(ap @ a @ ap, ap, atol=1e-10)
    assert np.allclose(ap, np.linalg.pinv(a, rcond=1e-10), atol=1e-10)


@pytest.mark.parametrize("form", [FORM_PUSH, FORM_PULL])
def test_isotropic_noise_coefficient_reproduces_the_scalar_variance(oracle_lib, form):
    r, n, q, dt = 3, 64, 0.37, 0.03
    lo, hi, x = _nodes(r, n, 0.8)
    m = _model(r, F_COS, q=q)
    s = (1.0, 2.0, 4.0)
    c = oracle.kernel_coefficients(s)
    lw = -np.random.default_rng(2).random(n) * 3
    ref, ncl = oracle.propagate_ex(m, s, c, x, lo, hi, dt, lw, form=form)
    ap, logdet, rank = oracle.noise_pinv(math.sqrt(q) * np.eye(r))
    got, ncl2 = oracle.propagate_ex(m, s, c, x, lo, hi, dt, lw, form=form, apinv=ap, logdet_a=logdet)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin) and ncl == ncl2 and rank == r
    assert np.allclose(got[fin], ref[fin], rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("form", [FORM_PUSH, FORM_PULL])
@pytest.mark.parametrize("rank", [4, 2])
def test_general_noise_single_source_against_scipy(oracle_lib, form, rank):
    """Invertible a: scipy's full-covariance Gaussian.  Singular a (rank < r): scipy's Gaussian in the
    coordinates of a's range, plus the constant the table keeps: (2 pi tau)^{-r/2} det_+(a)^{-1/2}."""
    r, n, dt = 4, 40, 0.05
    lo, hi, x = _nodes(r, n, 0.7)
    U, Q, lam = _random_U(r, rank, 5 + rank)
    ap, logdet, k = oracle.noise_pinv(U)
    assert k == rank
    m = _model(r, F_COS)
    F = oracle.drift(m, x)
    div = oracle.divergence(m, x)
    j0 = 11
    lw = np.full(n, -np.inf)
    lw[j0] = 0.0
    got, _ = oracle.propagate_ex(m, (1.0,), (1.0, 0.0), x, lo, hi, dt, lw, form=form, apinv=ap, logdet_a=logdet)
    logdV = np.sum(np.log(hi - lo)) - np.log(n)
    tau = dt
    for i in range(n):
        d = (x[j0] - x[i] + tau * F[i]) if form == FORM_PULL else (x[i] - x[j0] - tau * F[j0])
        if rank == r:
            ref = multivariate_normal.logpdf(d, np.zeros(r), tau * (U @ U.T))
        else:
            z = Q[:, :rank].T @ d
            ref = multivariate_normal.logpdf(z, np.zeros(rank), tau * np.diag(lam[:rank])) \
                - 0.5 * (r - rank) * math.log(2 * math.pi * tau)
        if form == FORM_PULL:
            ref -= tau * div[i]
        assert abs(got[i] - (logdV + ref)) <= 1e-11 * max(1.0, abs(ref)), (i, got[i], logdV + ref)


def test_general_noise_linearity_and_pseudo_inverse_invariance(oracle_lib):
    """The singular kernel ignores displacements along a's null space: moving every node along it
    leaves the prediction unchanged; and the sum is linear in the weights."""
    r, n, dt = 3, 48, 0.04
    U, Q, lam = _random_U(r, 2, 9)
    ap, logdet, _ = oracle.noise_pinv(U)
    lo, hi, x = _nodes(r, n, 0.6)
    m = _model(r, F_ZERO)
    s = (1.0, 2.0)
    c = oracle.kernel_coefficients(s)
    rng = np.random.default_rng(4)
    lw = -rng.random(n) * 2
    # displacements along the null direction of a do not enter the kernel: with the nodes moved along it
    # (and a box large enough to hold them), the pairwise sums are unchanged and a one-scale prediction
    # without identity term changes by the log ratio of the quadrature weights only
    shift = np.outer(rng.standard_normal(n) * 0.01, Q[:, 2])
    vol_ratio = np.sum(np.log(hi + 1 - (lo - 1))) - np.sum(np.log(hi - lo))
    one, _ = oracle.propagate_ex(m, (1.0,), (1.0, 0.0), x, lo, hi, dt, lw, apinv=ap, logdet_a=logdet)
    one_m, _ = oracle.propagate_ex(m, (1.0,), (1.0, 0.0), x + shift, lo - 1, hi + 1, dt, lw, apinv=ap,
                                   logdet_a=logdet)
    f1 = np.isfinite(one) & np.isfinite(one_m)
    assert f1.sum() > n // 2
    assert np.allclose(one_m[f1] - one[f1], vol_ratio, rtol=0, atol=1e-11)
    a = np.where(rng.random(n) < 0.5, -rng.random(n), -np.inf)
    b = np.where(rng.random(n) < 0.5, -rng.random(n), -np.inf)
    la, _ = oracle.propagate_ex(m, s, c, x, lo, hi, dt, a, apinv=ap, logdet_a=logdet)
    lb, _ = oracle.propagate_ex(m, s, c, x, lo, hi, dt, b, apinv=ap, logdet_a=logdet)
    lab, _ = oracle.propagate_ex(m, s, c, x, lo, hi, dt, np.logaddexp(a, b), apinv=ap, logdet_a=logdet)
    ok = np.isfinite(la) & np.isfinite(lb) & np.isfinite(lab)
    assert np.allclose(lab[ok], np.logaddexp(la[ok], lb[ok]), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rank", [3, 2])
def test_general_observation_noise_update(oracle_lib, rank):
    """Invertible b: the Gaussian likelihood ratio log N(dy; h dt, b dt) - log N(dy; 0, b dt) (scipy).
    Singular b: the same ratio in the coordinates of b's range, and invariance under null components."""
    r, n, dt = 3, 30, 0.01
    rng = np.random.default_rng(rank)
    V, Q, lam = _random_U(r, rank, 20 + rank)
    bp, _, k = oracle.noise_pinv(V)
    assert k == rank
    m = _model(r, F_ZERO, obs=H_CUBE)
    x = rng.standard_normal((n, r))
    dy = rng.standard_normal(r) * 0.1
    lw0 = rng.standard_normal(n)
    got = oracle.loglik_update_ex(m, x, dy, dt, bp, lw0)
    h = x ** 3
    for i in range(n):
        if rank == r:
            cov = dt * (V @ V.T)
            ref = multivariate_normal.logpdf(dy, h[i] * dt, cov) - multivariate_normal.logpdf(dy, np.zeros(r), cov)
        else:
            P = Q[:, :rank]
            cov = dt * np.diag(lam[:rank])
            ref = multivariate_normal.logpdf(P.T @ dy, P.T @ h[i] * dt, cov) - \
                multivariate_normal.logpdf(P.T @ dy, np.zeros(rank), cov)
        assert abs(got[i] - (lw0[i] + ref)) <= 1e-10 * max(1.0, abs(ref)), (i, got[i], lw0[i] + ref)
    if rank < r:
        moved = oracle.loglik_update_ex(m, x, dy + 0.3 * Q[:, -1], dt, bp, lw0)
        assert np.allclose(moved, got, rtol=1e-12, atol=1e-11)
    # b = rho2 I reproduces the isotropic update
    iso = oracle.OModel(r, r, F_ZERO, None, H_CUBE, None, 0.0, 1.0, 0.3)
    bp_iso, _, _ = oracle.noise_pinv(math.sqrt(0.3) * np.eye(r))
    assert np.allclose(oracle.loglik_update_ex(iso, x, dy, dt, bp_iso, lw0), oracle.loglik_update(iso, x, dy, dt, lw0),
                       rtol=1e-12, atol=1e-11)
