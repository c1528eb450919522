"""Longer runs against the FP64 oracle: 100 steps with discontinuities, boundaries and the
optional limiters, to show that the GPU path does not drift from the oracle beyond rounding.

Tolerance: 1e-12 * scale, as for the short parity runs: after 100 steps the measured
differences are below 1e-14 * scale (8e-14 at scales 11 and 22).  Counters (limiter
replacements, centre fallbacks, transonic flags) must match exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I
from test_gpu_shocks import _riemann_state

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(out, st, tol):
    scale = max(float(np.abs(st.avg).max()), float(np.abs(st.K).max()))
    d = {k: float(np.abs(out[k] - getattr(st, k)).max()) for k in ("avg", "K", "X", "Y")}
    _flush(f"  max differences {d} (scale {scale:.3g})")
    assert max(d.values()) < tol * scale, d


def test_shock_reflection_100_steps():
    _flush("[gpu] shock reflection 120x30, 100 steps, averaged linearisation")
    st = I.shock_reflection_state(120, 30)
    s = af.Solver.for_state(st, precision=0, linearisation=af.AF_LIN_AVG)
    t, n = s.run(1e9, 0.3, 100)
    out = s.get_state()
    s.close()
    e, n2, _ = oracle.run(st, 1e9, 0.3, max_steps=100, mode=oracle.MODE_AVG)
    assert e == 0 and n == n2 == 100
    assert abs(t - st.t) < 1e-12
    _compare(out, st, 1e-12)


def test_riemann_indicators_100_steps():
    _flush("[gpu] 2D Riemann data, 100 steps, limiter + Algorithm 2 + shock blend")
    st = _riemann_state()
    s = af.Solver.for_state(st, precision=0, linearisation=af.AF_LIN_AVG, limiter=True,
                            transonic=True, shock_limiter=True)
    t, n = s.run(1e9, 0.3, 100)
    out = s.get_state()
    cnt = s.counters()
    s.close()
    e, n2, c2 = oracle.run(st, 1e9, 0.3, max_steps=100, mode=oracle.MODE_AVG, limiter=True,
                           tsw=True, shock=True)
    assert e == 0 and n == n2 == 100
    for k in (0, 1, 2, 3, 5):
        assert cnt[k] == c2[k], (k, list(cnt), list(c2))
    _compare(out, st, 1e-12)
