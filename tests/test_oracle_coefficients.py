"""Pins of the multi-scale kernel coefficients (Sec. 4.3.2-4.3.3, V c = d)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_coefficients.txt")


def _golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            s, c = line.split(";")
            rows.append((np.array(s.split(), float), np.array(c.split(), float)))
    return rows


def test_printed_second_order_coefficients(oracle_lib):
    for s, c in _golden():
        assert np.allclose(oracle.kernel_coefficients(s), c, rtol=0, atol=1e-14)


def test_three_scale_closed_form(oracle_lib):
    # exact solution for s = {1, 2, 4} with mu = 3/2, 2 (derived symbolically)
    r2 = np.sqrt(2.0)
    expect = np.array([1 + r2, -8 - 6 * r2, 16 + 8 * r2, -8 - 3 * r2])
    assert np.allclose(oracle.kernel_coefficients([1, 2, 4]), expect, rtol=0, atol=1e-12)


def test_single_scale_is_the_first_order_kernel(oracle_lib):
    assert np.array_equal(oracle.kernel_coefficients([1.0]), [1.0, 0.0])


def test_scale_order_permutes_coefficients(oracle_lib):
    a = oracle.kernel_coefficients([1, 2, 4])
    b = oracle.kernel_coefficients([4, 1, 2])
    assert np.allclose(b, [a[2], a[0], a[1], a[3]], atol=1e-12)
