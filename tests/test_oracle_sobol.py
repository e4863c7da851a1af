"""Pins of the oracle's Sobol generator (Appendix A, Sobol sequence).

Independent references: the van der Corput closed form (bit reversal of the
Gray code), the Pascal-matrix generator of the second dimension, scipy's
unscrambled Sobol (Joe-Kuo numbers agree with ours in dimensions 1-2), the
count of primitive polynomials phi(2^s - 1)/s, and the net / stratification
properties that any digital (t, m, s)-net construction and its random linear
scrambles must keep.
"""
import math

import numpy as np
import pytest
from scipy.stats import qmc

import oracle


def bitrev32(v: int) -> int:
    return int(f"{v:032b}"[::-1], 2)


def test_dimension_one_is_van_der_corput_in_gray_order(oracle_lib):
    n = 4096
    codes = oracle.sobol_codes(1, n, 0, scramble=False)[:, 0]
    expect = np.array([bitrev32(i ^ (i >> 1)) for i in range(n)], dtype=np.uint32)
    assert np.array_equal(codes, expect)


def test_dimension_two_is_pascal_matrix(oracle_lib):
    v = oracle.sobol_directions(2)[1]
    for k in range(1, 33):  # direction number k, binary digits j = 1..32 (most significant first)
        digits = [(int(v[k - 1]) >> (32 - j)) & 1 for j in range(1, 33)]
        expect = [math.comb(k - 1, j - 1) % 2 if j <= k else 0 for j in range(1, 33)]
        assert digits == expect, k


def test_first_two_dimensions_match_scipy(oracle_lib):
    n = 2048
    ref = qmc.Sobol(d=2, scramble=False, bits=32).random(n)
    got = oracle.sobol_codes(2, n, 0, scramble=False).astype(np.float64) / 2.0**32
    assert np.array_equal(ref, got)


def test_first_index_offsets_the_sequence(oracle_lib):
    full = oracle.sobol_codes(5, 300, 0, scramble=True, seed=3)
    tail = oracle.sobol_codes(5, 100, 200, scramble=True, seed=3)
    assert np.array_equal(full[200:], tail)


def _totient(N: int) -> int:
    res, m, p = N, N, 2
    while p * p <= m:
        if m % p == 0:
            while m % p == 0:
                m //= p
            res -= res // p
        p += 1
    if m > 1:
        res -= res // m
    return res


def test_primitive_polynomial_counts(oracle_lib):
    idx = 0
    for s in range(1, 12):
        count = _totient(2**s - 1) // s
        degs = [oracle.primitive_poly(idx + t)[0] for t in (0, count - 1, count)]
        assert degs[0] == s and degs[1] == s and degs[2] == s + 1, (s, degs)
        idx += count


def test_direction_numbers_are_odd_and_bounded(oracle_lib):
    v = oracle.sobol_directions(300).astype(np.uint64)
    for k in range(1, 33):
        col = v[:, k - 1]
        assert np.all((col >> np.uint64(32 - k)) & np.uint64(1) == 1)          # m_k odd
        assert np.all(col & np.uint64((1 << (32 - k)) - 1) == 0)               # m_k < 2^k


@pytest.mark.parametrize("scramble", [False, True])
def test_first_two_dimensions_form_a_0m2_net(oracle_lib, scramble):
    m = 10
    codes = oracle.sobol_codes(2, 2**m, 0, scramble=scramble, seed=11).astype(np.int64)
    for p in range(m + 1):
        q = m - p
        cell = (codes[:, 0] >> (32 - p)) * (2**q) + (codes[:, 1] >> (32 - q)) if p < 32 else None
        assert len(np.unique(cell)) == 2**m, (p, q)


@pytest.mark.parametrize("scramble", [False, True])
def test_every_dimension_is_dyadically_stratified(oracle_lib, scramble):
    m, r = 9, 400
    codes = oracle.sobol_codes(r, 2**m, 0, scramble=scramble, seed=5).astype(np.int64)
    top = codes >> (32 - m)
    for d in range(r):
        assert len(np.unique(top[:, d])) == 2**m, d


def test_scramble_is_keyed_by_seed(oracle_lib):
    a = oracle.sobol_codes(8, 64, 0, scramble=True, seed=1)
    b = oracle.sobol_codes(8, 64, 0, scramble=True, seed=1)
    c = oracle.sobol_codes(8, 64, 0, scramble=True, seed=2)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_scrambled_points_have_low_discrepancy(oracle_lib):
    n, r = 1024, 6
    pts = oracle.sobol_codes(r, n, 0, scramble=True, seed=7).astype(np.float64) / 2.0**32
    rnd = np.random.default_rng(0).random((n, r))
    assert qmc.discrepancy(pts) < 0.25 * qmc.discrepancy(rnd)


def test_code_to_box_map(oracle_lib):
    lo, hi = np.array([-1.5, 0.25]), np.array([2.5, 0.75])
    codes = np.array([[0, 0], [2**31, 2**31], [2**32 - 1, 2**30]], dtype=np.uint32)
    x = oracle.codes_to_points(codes, lo, hi)
    assert np.array_equal(x[0], lo)                          # code 0 is the lower face
    assert np.array_equal(x[1], 0.5 * (lo + hi))             # code 2^31 is the centre
    assert np.all(x[2] < hi) and x[2, 1] == 0.375
    assert oracle.is_boundary(x, lo, hi).tolist() == [True, False, False]
