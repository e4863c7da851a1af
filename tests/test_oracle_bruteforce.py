"""Brute-force pins of the oracle: the multi-scale prediction as a 50-digit double sum, its second-order
consistency, SplitMix64's published outputs, resampling by exhaustive search and the restart map as a
translation.

* Prediction (Sec. 4.3.3, eq. general_kernel; quadrature of Sec. 4.1 with weight vol(box)/n; Dirichlet
  rows of Sec. 4.2): for n <= 64 the push-form sum
      sum_s c_s dV sum_j prod_k N(x_ik; x_jk + tau_s f_k(x_j), q tau_s) e^{l_j} + c_{S+1} e^{l_i}
  is formed in the linear domain with mpmath at 50 digits, one-dimensional normal densities multiplied
  coordinate by coordinate, and the coefficients in the closed forms the paper prints (alpha, beta, gamma
  of Theorem thm:2ndorderkernel) or that its constraints give exactly for scales {1, 2, 4}.  None of the
  oracle's log-domain arithmetic (maxima, shifts, sign bookkeeping) appears on this side.
* Second-order consistency: with scales {1, 2, 4} the constraints of Sec. 4.3.3 also remove the dt^2 term
  of the push kernel's expansion (whose error terms are integer powers of dt, the Gaussian's odd moments
  vanishing), so (L u - u)/dt - L* u falls like dt^2; with one scale like dt.
* SplitMix64 (Steele, Lea & Flood 2014): the published reference outputs for seeds 0 and 1234567.
* Resampling: the integer systematic positions evaluated with Python's exact integers and the ancestors
  found by scanning the prefix sums from the start for every position (O(n^2)).
* Restart (Sec. 6): the new node set is the pre-generated reference set translated by the estimate.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import F_COS, F_LINEAR, F_ZERO, H_IDENTITY


def _coefficients(S):
    """Closed forms: S = 1 -> (1, 0); S = 2 -> the printed alpha, beta, gamma; S = 3 -> exact for {1,2,4}."""
    with mpmath.workdps(50):
        r2 = mpmath.sqrt(2)
        if S == 1:
            return (1.0,), [mpmath.mpf(1), mpmath.mpf(0)]
        if S == 2:
            return (1.0, 2.0), [-r2 - 1, 4 + 2 * r2, -2 - r2]
        return (1.0, 2.0, 4.0), [1 + r2, -8 - 6 * r2, 16 + 8 * r2, -8 - 3 * r2]


def _drift_mp(kind, A, xj):
    if kind == F_ZERO:
        return [mpmath.mpf(0)] * len(xj)
    if kind == F_COS:
        return [mpmath.cos(v) for v in xj]
    return [mpmath.fsum(mpmath.mpf(A[k, l]) * xj[l] for l in range(len(xj))) for k in range(len(xj))]


def _brute_force(kind, A, x, lw, lo, hi, dt, q, scales, c):
    """Returns per target: (value or None for -inf, clamped flag, sum of absolute terms / |sum|)."""
    n, r = x.shape
    out = []
    with mpmath.workdps(50):
        X = [[mpmath.mpf(float(v)) for v in row] for row in x]
        bnd = [any(abs(x[i, k] - lo[k]) <= 1e-12 or abs(hi[k] - x[i, k]) <= 1e-12 for k in range(r))
               for i in range(n)]
        vol = mpmath.fprod(mpmath.mpf(float(hi[k])) - mpmath.mpf(float(lo[k])) for k in range(r))
        dV = vol / n
        F = [_drift_mp(kind, A, X[j]) for j in range(n)]
        E = [mpmath.e ** mpmath.mpf(float(v)) if np.isfinite(v) else mpmath.mpf(0) for v in lw]
        for i in range(n):
            if bnd[i]:
                out.append((None, False, 0))
                continue
            total, absum = mpmath.mpf(0), mpmath.mpf(0)
            for s, cs in zip(scales, c[:-1]):
                tau = mpmath.mpf(dt) / s
                sd = mpmath.sqrt(mpmath.mpf(q) * tau)
                acc = mpmath.mpf(0)
                for j in range(n):
                    if bnd[j] or E[j] == 0:
                        continue
                    dens = mpmath.fprod(mpmath.npdf(X[i][k], X[j][k] + tau * F[j][k], sd) for k in range(r))
                    acc += dens * E[j]
                total += cs * dV * acc
                absum += abs(cs) * dV * acc
            total += c[-1] * E[i]
            absum += abs(c[-1]) * E[i]
            if absum == 0:
                out.append((None, False, 0))
            elif total <= 0:
                out.append((None, True, 0))
            else:
                out.append((float(mpmath.log(total)), False, float(absum / total)))
    return out


CASES = {
    # name: (r, n, half-width, q, dt, drift)
    "r1": (1, 64, 1.0, 0.5, 0.05, None),
    "r3": (3, 64, 1.0, 1.0, 0.09, None),
}


@pytest.mark.parametrize("S", [1, 2, 3])
@pytest.mark.parametrize("drift", [F_ZERO, F_COS, F_LINEAR])
@pytest.mark.parametrize("case", sorted(CASES))
def test_prediction_equals_50_digit_double_sum(oracle_lib, case, drift, S):
    r, n, half, q, dt, _ = CASES[case]
    lo, hi = -half * np.ones(r), half * np.ones(r)
    # unscrambled points from index 0: point 0 is the corner lo (a boundary node)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 0, False), lo, hi)
    rng = np.random.default_rng(100 * r + 10 * drift + S)
    lw = -3.0 * rng.random(n)
    lw[[5, 11]] = -np.inf
    lw[0] = 2.0                      # weight on the boundary node: must not contribute
    lw[n // 2] = 4.0                 # one heavy source: far targets get a negative signed sum for S > 1
    A = rng.standard_normal((r, r)) * 0.5 - np.eye(r)
    model = oracle.OModel(r, r, drift, A if drift == F_LINEAR else None, H_IDENTITY, None, 0.0, q, 1.0)
    scales, c_mp = _coefficients(S)
    c = np.array([float(v) for v in c_mp])
    got, nclamped = oracle.propagate(model, scales, c, x, lo, hi, dt, lw)
    ref = _brute_force(drift, A, x, lw, lo, hi, dt, q, scales, c_mp)
    assert got[0] == -np.inf and ref[0][0] is None
    n_ref_clamped = 0
    for i, (val, clamped, cond) in enumerate(ref):
        n_ref_clamped += clamped
        if val is None:
            assert got[i] == -np.inf, (i, got[i], clamped)
            continue
        tol = 1e-13 * max(1.0, abs(val)) + 4e-16 * cond
        assert abs(got[i] - val) <= tol, (i, got[i], val, cond)
    assert nclamped == n_ref_clamped
    if S > 1 and case == "r1":
        assert n_ref_clamped > 0   # the case exercises the clamp of a negative combination


def test_linearity_in_the_weights_with_three_signed_scales(oracle_lib):
    """exp(L(a (+) b)) = exp(L a) + exp(L b) on every row where none of the three sums is clamped."""
    r, n, q, dt = 2, 64, 1.0, 0.05
    lo, hi = -np.ones(r), np.ones(r)
    x = oracle.codes_to_points(oracle.sobol_codes(r, n, 1, True, 4), lo, hi)
    model = oracle.OModel(r, r, F_COS, None, H_IDENTITY, None, 0.0, q, 1.0)
    s = (1.0, 2.0, 4.0)
    c = oracle.kernel_coefficients(s)
    rng = np.random.default_rng(8)
    a = np.where(rng.random(n) < 0.5, -rng.random(n), -np.inf)
    b = np.where(rng.random(n) < 0.5, 1.0 - rng.random(n), -np.inf)
    la, _ = oracle.propagate(model, s, c, x, lo, hi, dt, a)
    lb, _ = oracle.propagate(model, s, c, x, lo, hi, dt, b)
    lab, _ = oracle.propagate(model, s, c, x, lo, hi, dt, np.logaddexp(a, b))
    ok = np.isfinite(la) & np.isfinite(lb) & np.isfinite(lab)
    assert ok.sum() > n // 2
    assert np.allclose(lab[ok], np.logaddexp(la[ok], lb[ok]), rtol=1e-12, atol=1e-12)
    # scaling every weight by e^t adds t to every row
    l2, _ = oracle.propagate(model, s, c, x, lo, hi, dt, np.logaddexp(a, b) + 7.5)
    assert np.allclose(l2[ok] - lab[ok], 7.5, rtol=0, atol=1e-11)


def test_three_scales_are_second_order_consistent(oracle_lib):
    """(L u - u)/dt - L* u shrinks like dt^2 with scales {1,2,4} and like dt with one scale (Theorem
    thm:2ndorderkernel and Sec. 4.3.3: the constraints match the dt term and remove the next orders)."""
    n = 4096
    lo, hi = np.array([-5.0]), np.array([5.0])
    x = oracle.codes_to_points(oracle.sobol_codes(1, n, 0, False), lo, hi)[:, 0]
    mu, sd = 0.3, 0.5
    u = np.exp(-0.5 * ((x - mu) / sd) ** 2) / (sd * np.sqrt(2 * np.pi))
    du = -(x - mu) / sd**2 * u
    d2u = ((x - mu) ** 2 / sd**4 - 1 / sd**2) * u
    Lstar = 0.5 * d2u - (-np.sin(x) * u + np.cos(x) * du)      # f = cos, q = 1
    model = oracle.OModel(1, 1, F_COS, None, H_IDENTITY, None, 0.0, 1.0, 1.0)
    inner = np.abs(x - mu) < 1.5
    rates = {}
    for scales in ((1.0,), (1.0, 2.0, 4.0)):
        c = oracle.kernel_coefficients(scales)
        errs = []
        for dt in (0.04, 0.02, 0.01):
            out, _ = oracle.propagate(model, scales, c, x[:, None], lo, hi, dt, np.log(u))
            errs.append(np.max(np.abs((np.exp(out) - u) / dt - Lstar)[inner]))
        rates[len(scales)] = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates[1] > 0.85) and np.all(rates[1] < 1.2), rates
    assert np.all(rates[3] > 1.8) and np.all(rates[3] < 2.3), rates


def test_splitmix64_published_outputs(oracle_lib):
    # reference outputs of the SplitMix64 generator (Steele, Lea & Flood 2014) started at state 0 and
    # at state 1234567, as published with its reference implementation and common test vectors
    assert [oracle.splitmix64_at(0, k) for k in range(5)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [oracle.splitmix64_at(1234567, k) for k in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]


def _naive_resample(w, seed, step):
    n = len(w)
    Wi = [int(math.floor(max(v, 0.0) * 2.0**53)) for v in w]   # w * 2^53 is exact in FP64
    C, run = [], 0
    for v in Wi:
        run += v
        C.append(run)
    W = run
    U = oracle.splitmix64_at(oracle.splitmix64_at(seed, 2), step) >> 32
    idx = []
    for t in range(n):
        P = ((t << 32) + U) * W // (n << 32)
        i = 0
        while not C[i] > P:     # the first index whose prefix sum exceeds the position
            i += 1
        idx.append(i)
    return np.array(idx, dtype=np.int64)


@pytest.mark.parametrize("kind", ["random", "one_hot", "zeros_at_ends", "single", "tiny_and_huge"])
def test_resampling_equals_exhaustive_search(oracle_lib, kind):
    rng = np.random.default_rng(21)
    n = 1 if kind == "single" else 301
    if kind == "random":
        w = rng.random(n) ** 3
    elif kind == "one_hot":
        w = np.zeros(n); w[137] = 1.0
    elif kind == "zeros_at_ends":
        w = rng.random(n); w[:40] = 0.0; w[-55:] = 0.0
    elif kind == "single":
        w = np.ones(1)
    else:
        w = np.full(n, 1e-17); w[::7] = rng.random(len(w[::7]))
    w = w / w.sum()
    for seed, step in ((0, 1), (3, 2), (77, 40)):
        got = oracle.resample(w, seed, step)
        assert np.array_equal(got, _naive_resample(w, seed, step)), (kind, seed, step)


def test_restart_translates_the_reference_set(oracle_lib):
    """Sec. 6: one reference set in [-R, R]^r translated by the estimate at every restart, so the new
    nodes minus the estimate are the reference nodes, and their mean is the estimate plus the reference
    set's mean offset."""
    r, n, R = 5, 512, 0.3
    codes = oracle.sobol_codes(r, n, 0, True, 9)
    _, _, x0, _ = oracle.restart_nodes(codes, np.zeros(r), R)
    ref_offset = x0.mean(axis=0)
    for mean in (np.array([0.5, -1.25, 2.0, 0.0, 100.0]), np.array([-3.0, 1e-3, 7.5, -0.25, 1.0])):
        lo, hi, x, _ = oracle.restart_nodes(codes, mean, R)
        eps = 4 * np.finfo(float).eps * (np.abs(mean) + R)
        assert np.all(np.abs((x - mean) - x0) <= eps)
        # the mean itself carries the summation rounding of 512 values of size |mean| + R
        assert np.all(np.abs(x.mean(axis=0) - (mean + ref_offset)) <= 16 * eps)
        assert np.all(np.abs(x0) <= R)
