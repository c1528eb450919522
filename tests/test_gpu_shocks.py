"""Algorithm 2 (transonic-shock linearisation) and the shock-indicator blend of Sec. 3.4 on the
GPU: parity with the FP64 oracle (values and counters) on a moving transonic shock, a
four-state 2D Riemann configuration and the shock-reflection grid with walls and inflow; the
transonic shock's speed; option errors.

Tolerances as in the other parity tests: FP64 1e-12 * scale, FP32 bulk 1e-6 * scale.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I
from test_oracle_shocks import _jump_state, _position, _shock_pair

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _assert_close(out, ref, tol, label=""):
    scale = max(float(np.abs(ref.avg).max()), float(np.abs(ref.K).max()))
    d = {k: float(np.abs(out[k] - getattr(ref, k)).max()) for k in ("avg", "K", "X", "Y")}
    print(f"    {label}: achieved max|diff|/scale {max(d.values()) / scale:.3e} (gate {tol:g})",
          flush=True)
    bad = {k: v for k, v in d.items() if v > tol * scale}
    assert not bad, f"{label}: {d} (tol {tol * scale:.3e})"


# Four constant states (lower left, lower right, upper left, upper right) whose flows collide:
# across every dividing line u - c (v - c) goes from positive to negative, so every line
# carries a transonic shock.
RIEMANN_STATES = (np.array([1.0, 1.3, 1.3, 0.7]), np.array([1.8, -0.1, 1.3, 2.0]),
                  np.array([1.8, 1.3, -0.1, 2.0]), np.array([2.5, -0.2, -0.2, 3.0]))


def _riemann_state(n=44, m=38):
    """RIEMANN_STATES meeting at (0.55, 0.45) of [0,1]^2, outflow on every side.  Point values
    on the dividing lines take the mean of the adjacent states."""
    states = RIEMANN_STATES
    grid = I.Grid(n, m, 0.0, 1.0, 0.0, 1.0, I.BC_OUTFLOW, I.BC_OUTFLOW)
    xs, ys = 0.55, 0.45

    def prim(x, y, sites):
        W = np.zeros((4,) + x.shape)
        right, top = x > xs, y > ys
        for q, (r, t) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
            sel = (right == bool(r)) & (top == bool(t))
            W[:, sel] = states[q][:, None]
        return W

    avg = I.cell_average(lambda x, y: prim(x, y, False), grid, I.GAMMA, 4)
    st = I.State(grid, I.GAMMA, avg, prim(*grid.k_sites(), True), prim(*grid.x_sites(), True),
                 prim(*grid.y_sites(), True))
    return st


CASES = {
    "transonic_shock": lambda: _jump_state(*_shock_pair(1.3, -0.2), nx=60, ny=5),
    "riemann_2d": _riemann_state,
    "shock_reflection": lambda: I.shock_reflection_state(120, 30),
}


@pytest.mark.parametrize("tsw,shock", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("case", list(CASES))
def test_indicators_match_oracle_fp64(case, tsw, shock):
    _flush(f"[gpu] indicators {case} tsw={tsw} shock={shock} fp64, 12 steps")
    st = CASES[case]()
    s = af.Solver.for_state(st, precision=0, linearisation=af.AF_LIN_AVG, limiter=True,
                            transonic=tsw, shock_limiter=shock)
    t, n = s.run(1e9, 0.3, 12)
    out = s.get_state()
    cnt = s.counters()
    s.close()
    e, n2, c2 = oracle.run(st, 1e9, 0.3, max_steps=12, mode=oracle.MODE_AVG, limiter=True,
                           tsw=tsw, shock=shock)
    assert e == 0 and n == n2 == 12
    assert abs(t - st.t) < 1e-13
    _assert_close(out, st, 1e-12, f"{case} tsw {tsw} shock {shock}")
    for k in (0, 1, 2, 3, 5):
        assert cnt[k] == c2[k], (k, list(cnt), list(c2))
    if tsw and case != "shock_reflection":
        assert cnt[af.AF_CNT_TSW] > 0


@pytest.mark.parametrize("mode", [af.AF_LIN_AF3, af.AF_LIN_SIMPLE])
def test_indicators_in_other_modes_match_oracle(mode):
    _flush(f"[gpu] indicators riemann mode={mode}")
    st = _riemann_state()
    s = af.Solver.for_state(st, precision=0, linearisation=mode, limiter=True, transonic=True,
                            shock_limiter=True)
    s.run(1e9, 0.3, 8)
    out = s.get_state()
    s.close()
    e, _, _ = oracle.run(st, 1e9, 0.3, max_steps=8, mode=mode, limiter=True, tsw=True,
                         shock=True)
    assert e == 0
    _assert_close(out, st, 1e-12, f"mode {mode}")


@pytest.mark.parametrize("case", list(CASES))
def test_indicators_fp32_bulk(case):
    _flush(f"[gpu] indicators {case} fp32")
    st = CASES[case]()
    s = af.Solver.for_state(st, precision=1, linearisation=af.AF_LIN_AVG, limiter=True,
                            transonic=True, shock_limiter=True)
    s.run(1e9, 0.3, 8)
    out = s.get_state()
    s.close()
    e, _, _ = oracle.run(st, 1e9, 0.3, max_steps=8, mode=oracle.MODE_AVG, limiter=True,
                         tsw=True, shock=True)
    assert e == 0
    _assert_close(out, st, 1e-6, f"{case} fp32")


@pytest.mark.parametrize("prec", [0, 1])
def test_transonic_shock_speed_on_gpu(prec):
    """The left-moving transonic shock (Mach 1.3, speed -0.2) to t = 0.6 on 100 x 4 cells:
    with Algorithm 2 within half a cell of its exact position, one corner line flagged per
    step; without it the shock stalls (the oracle's pin, on the GPU)."""
    _flush(f"[gpu] transonic shock speed prec={prec}")
    L, R = _shock_pair(1.3, -0.2)
    pos = {}
    for tsw in (False, True):
        st = _jump_state(L, R)
        s = af.Solver.for_state(st, precision=prec, linearisation=af.AF_LIN_AVG, limiter=True,
                                transonic=tsw)
        t, n = s.run(0.6, 0.3)
        out = s.get_state()
        cnt = s.counters()
        s.close()
        assert t == 0.6
        st.avg = out["avg"]
        pos[tsw] = _position(st, L, R)[0]
        if tsw:
            assert cnt[af.AF_CNT_TSW] == 16 * n
    assert abs(pos[True] + 0.12) < 0.01
    assert abs(pos[False] + 0.12) > 0.04


def test_indicator_options():
    _flush("[gpu] indicator options")
    st = _riemann_state(16, 12)
    s = af.Solver.for_state(st, limiter=True)
    assert s.get_option(af.AF_OPT_TRANSONIC) == 0
    s.set_option(af.AF_OPT_TRANSONIC, 1)
    s.set_option(af.AF_OPT_SHOCK_LIMITER, 1)
    assert s.get_option(af.AF_OPT_TRANSONIC) == 1
    assert s.get_option(af.AF_OPT_SHOCK_LIMITER) == 1
    with pytest.raises(af.AfError):
        s.set_option(af.AF_OPT_SHOCK_LIMITER, 2)
    # switching off restores the plain method bit for bit
    s.set_option(af.AF_OPT_TRANSONIC, 0)
    s.set_option(af.AF_OPT_SHOCK_LIMITER, 0)
    s.run(1e9, 0.3, 3)
    a = s.get_state()
    s.close()
    s2 = af.Solver.for_state(st, limiter=True)
    s2.run(1e9, 0.3, 3)
    b = s2.get_state()
    s2.close()
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_indicators_equal_single_handles(prec):
    """Batched grids with both indicators on (uneven sizes, outflow, walls and inflow) give
    the single-grid results bit for bit."""
    _flush(f"[gpu] batched indicators prec={prec}")
    states = [_riemann_state(), CASES["transonic_shock"](), I.shock_reflection_state(48, 12),
              _riemann_state(19, 23)]
    kw = dict(precision=prec, linearisation=af.AF_LIN_AVG, limiter=True, transonic=True,
              shock_limiter=True)
    b = af.BatchSolver.for_states(states, **kw)
    b.run(1e9, 0.3, 10)
    cb = b.counters()
    tot = np.zeros(8, dtype=np.int64)
    for g, st in enumerate(states):
        s = af.Solver.for_state(st, **kw)
        s.run(1e9, 0.3, 10)
        ref = s.get_state()
        tot += s.counters()
        s.close()
        out = b.get_state(g)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], ref[k]), (g, k)
    assert cb[af.AF_CNT_TSW] == tot[af.AF_CNT_TSW] > 0
    b.close()
