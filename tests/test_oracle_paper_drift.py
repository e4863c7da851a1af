"""The oracle's drift of the paper's large-scale test (Sec. 11, eq. A&A1):
f(x) = sin(x) (A x) + sin(2x) (A1 x) elementwise, A = bidiag(-0.5 | 0.1 above),
A1 = bidiag(-0.3 | 0.3 above), pinned by values that follow from exact sines."""
import math

import numpy as np

import oracle


def _f(x):
    m = oracle.OModel(len(x), len(x), oracle.F_PAPER_SINMIX, None, oracle.H_CUBE, None, 100.0, 1.0, 1.0)
    return oracle.drift(m, np.asarray(x, dtype=np.float64)[None, :])[0]


def test_vanishes_where_both_sines_vanish():
    # sin(k pi) = sin(2 k pi) = 0 for every coordinate, whatever A x and A1 x are
    x = math.pi * np.array([1.0, -2.0, 3.0, 1.0, -1.0])
    assert np.max(np.abs(_f(x))) < 1e-13


def test_single_coordinate_at_half_pi():
    # x = pi/2 e_k: sin(x_k) = 1 and sin(2 x_k) = 0, so f_k = -0.5 pi/2 (the diagonal of A); every other
    # coordinate has sin(x_j) = 0; this holds at the last coordinate too, which has no superdiagonal term
    for r, k in ((6, 0), (6, 3), (6, 5), (1, 0)):
        x = np.zeros(r)
        x[k] = math.pi / 2
        f = _f(x)
        assert abs(f[k] + math.pi / 4) < 1e-15
        assert np.all(np.delete(f, k) == 0.0)


def test_superdiagonal_couples_the_next_coordinate():
    # x_0 = pi/6 (sin = 1/2, sin 2x = sqrt(3)/2), x_1 = 1: f_0 picks up 0.1 x_1 (A) and 0.3 x_1 (A1); a
    # subdiagonal (lower bidiagonal A, A1) would leave f_0 without x_1 and give f_1 the x_0 terms instead
    x = np.array([math.pi / 6, 1.0, 0.0, 0.0])
    f = _f(x)
    f0 = 0.5 * (-0.5 * math.pi / 6 + 0.1) + math.sqrt(3) / 2 * (-0.3 * math.pi / 6 + 0.3)
    f1 = math.sin(1.0) * (-0.5) + math.sin(2.0) * (-0.3)
    assert abs(f[0] - f0) < 1e-15 and abs(f[1] - f1) < 1e-15
    assert f[2] == 0.0 and f[3] == 0.0
    # changing x_2 moves f_1 and f_2 only
    y = x.copy()
    y[2] = 0.7
    g = _f(y)
    assert g[0] == f[0] and g[3] == f[3] and g[1] != f[1] and g[2] != f[2]
