"""Host-side checks of the C ABI: the library loads, exports every declared call, and its
host-only logic (coefficients by Cramer's rule) agrees with the paper.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "yy.h")
LIB = os.path.join(ROOT, "paper_2509_16896_amd", "libyy.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:yy_status|const char\*)\s+(yy_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2509_16896_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_abi():
    from paper_2509_16896_amd import yy
    assert sorted(yy.EXPORTED) == _declared()
    for name in _declared():
        if name != "yy_last_error":
            assert callable(getattr(yy, name))


def test_cramer_coefficients_match_printed_values(lib):
    from paper_2509_16896_amd import yy
    c = yy.yy_kernel_coefficients([1.0, 2.0])
    assert np.allclose(c, [-np.sqrt(2) - 1, 4 + 2 * np.sqrt(2), -2 - np.sqrt(2)], rtol=0, atol=1e-13)
    r2 = np.sqrt(2.0)
    c3 = yy.yy_kernel_coefficients([1.0, 2.0, 4.0])
    assert np.allclose(c3, [1 + r2, -8 - 6 * r2, 16 + 8 * r2, -8 - 3 * r2], rtol=0, atol=1e-11)


def test_argument_errors_are_reported(lib):
    from paper_2509_16896_amd import yy
    with pytest.raises(yy.YYError) as ei:
        yy.yy_kernel_coefficients([1.0, 1.0])   # repeated scales make V singular
    assert ei.value.status == yy.YY_ERR_ARG
    with pytest.raises(yy.YYError):
        yy.yy_kernel_coefficients([1.0, -2.0])
    rc = lib.yy_create(None, 0, None)
    assert rc == yy.YY_ERR_ARG
