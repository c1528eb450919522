"""The FP64 arcsine table of the evolution operators' arc angles (kAsinC in af_device.hpp):
asin(x) = x + x^3 g(x^2) on [0, 1/sqrt(2)], g a polynomial of degree 18.  The table in the
header is checked against the arcsine in 40-digit arithmetic: with its coefficients as stored
and the polynomial evaluated exactly, the result is within a quarter of an ulp of asin(x)
everywhere on the interval (sampled densely, end points included)."""
import os
import re

import pytest

mp = pytest.importorskip("mpmath")

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2508_06273_amd", "csrc",
                   "af_device.hpp")


def _table():
    text = open(HDR).read()
    m = re.search(r"constexpr double kAsinC\[(\d+)\] = \{([^}]*)\};", text)
    assert m, "kAsinC not found"
    vals = [float(v) for v in m.group(2).replace("\n", " ").split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return vals


def test_asin_table_within_a_quarter_ulp():
    mp.mp.dps = 40
    coef = [mp.mpf(c) for c in _table()]
    xmax = mp.sqrt(mp.mpf(1) / 2)
    worst = mp.mpf(0)
    n = 3000
    for k in range(n + 1):
        x = xmax * k / n if k else mp.mpf(2) ** -30
        t = x * x
        p = mp.mpf(0)
        for a in reversed(coef):
            p = p * t + a
        y = mp.asin(x)
        ulp = mp.mpf(2) ** (mp.floor(mp.log(y, 2)) - 52)
        worst = max(worst, abs(x + x ** 3 * p - y) / ulp)
    assert worst < 0.25, float(worst)


def test_asin_table_leading_terms_are_the_series():
    """Near 0 the interpolant agrees with the Maclaurin series asin x = x + x^3/6 + 3x^5/40 +
    ...: the first coefficients are 1/6 and 3/40 up to the interpolation error."""
    c = _table()
    assert abs(c[0] - 1 / 6) < 1e-15
    assert abs(c[1] - 3 / 40) < 1e-12
