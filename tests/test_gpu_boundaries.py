"""Solid-wall and inflow boundaries (Sec. 4.3) on the GPU: parity with the FP64 oracle on
grids with several tiles and ragged edges, the batched path, argument errors, and the
shock-reflection problem run to t = 6 against the exact states of the regular reflection.

Tolerances as in the other parity tests: FP64 1e-12 * scale, FP32 bulk 1e-6 * scale.
"""
import math
import sys

import numpy as np
import pytest

import exact_shock as ES
import oracle
from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")

WALL, INFLOW, OUTFLOW, PER = I.BC_WALL, I.BC_INFLOW, I.BC_OUTFLOW, I.BC_PERIODIC


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


def _mixed_inflow_state():
    """Fourier data on a ragged grid with every kind of side: inflow left, wall right,
    outflow bottom, wall top; the inflow state is subsonic."""
    grid = I.Grid(27, 19, 0.0, 1.2, 0.0, 0.9, sides=(INFLOW, WALL, OUTFLOW, WALL),
                  inflow=((1.1, 0.4, 0.05, 0.95), None, None, None))
    return I.fourier_state(I.SEED_BASE + 6500, grid, I.GAMMA, 3)


CASES = {
    "box": lambda: I.box_state(29, seed=I.SEED_BASE + 6600, ny=21),
    "box_xwall_yper": lambda: I.box_state(17, seed=I.SEED_BASE + 6700, sides=(2, 2, 0, 0),
                                          ny=24),
    "box_xper_ywall": lambda: I.box_state(18, seed=I.SEED_BASE + 6800, sides=(0, 0, 2, 2),
                                          ny=11),
    "mixed_inflow": _mixed_inflow_state,
    "shock_reflection": lambda: I.shock_reflection_state(120, 30),
}


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", list(CASES))
def test_boundaries_match_oracle_fp64(case, mode):
    _flush(f"[gpu] boundaries {case} mode={mode} fp64, 6 steps")
    st = CASES[case]()
    s = af.Solver.for_state(st, precision=0, linearisation=mode)
    t, n = s.run(1e9, 0.3, 6)
    out = s.get_state()
    s.close()
    e, n2, _ = oracle.run(st, 1e9, 0.3, max_steps=6, mode=mode)
    assert e == 0 and n == n2 == 6
    assert abs(t - st.t) < 1e-13
    _assert_close(out, st, 1e-12, f"{case} mode {mode}")


@pytest.mark.parametrize("case", ["box", "mixed_inflow", "shock_reflection"])
def test_boundaries_match_oracle_fp32_bulk(case):
    _flush(f"[gpu] boundaries {case} fp32, 6 steps")
    st = CASES[case]()
    s = af.Solver.for_state(st, precision=1)
    s.run(1e9, 0.3, 6)
    out = s.get_state()
    s.close()
    e, _, _ = oracle.run(st, 1e9, 0.3, max_steps=6)
    assert e == 0
    _assert_close(out, st, 1e-6, f"{case} fp32")


def _wall_rarefaction_state():
    """Thin gas leaving the right wall at 4 (Mach ~7) behind a layer of one cell in which the
    velocity falls to zero at the wall: the near-vacuum that opens at the wall drives point
    values negative (inflow left, wall right and top, outflow bottom)."""
    grid = I.Grid(27, 19, 0.0, 1.2, 0.0, 0.9, sides=(INFLOW, WALL, OUTFLOW, WALL),
                  inflow=((1.1, 0.4, 0.05, 0.95), None, None, None))

    def fn(x, y):
        s = 0.5 * (1 + np.tanh((x - 0.9) / 0.05))
        w = np.tanh(np.maximum(1.2 - x, 0.0) / 0.03)
        return np.stack([1.0 - 0.9 * s, 0.3 * (1 - s) - 4.0 * s * w,
                         0.1 * np.sin(2 * np.pi * y / 0.9) * (1 - s), 1.0 - 0.97 * s])
    st = I.state_from_field(fn, grid, I.GAMMA, 3)
    st.K[1, :, -1] = 0.0
    st.X[1, :, -1] = 0.0
    return st


@pytest.mark.parametrize("mode,prec", [(1, 0), (0, 0), (1, 1)])
def test_boundaries_with_limiter_match_oracle(mode, prec):
    """Algorithm 3 next to a wall: without the limiter the run fails; with it, EG1 on
    piecewise constant data replaces point values at and near the wall, and the GPU matches
    the oracle, counters included (FP64)."""
    _flush(f"[gpu] wall rarefaction with limiter mode={mode} prec={prec}")
    st = _wall_rarefaction_state()
    s = af.Solver.for_state(st, precision=prec, linearisation=mode, limiter=True)
    t, n = s.run(1e9, 0.3, 7)
    out = s.get_state()
    cnt = s.counters()
    s.close()
    e, n2, c2 = oracle.run(st, 1e9, 0.3, max_steps=7, mode=mode, limiter=True)
    assert e == 0 and n == n2 == 7
    assert c2[0] > 0
    if prec == 0:
        assert list(cnt[:4]) == list(c2[:4])
        _assert_close(out, st, 1e-12, "limiter")
    else:
        assert cnt[0] > 0
        _assert_close(out, st, 1e-6, "limiter fp32")


def test_batched_boundaries_equal_single_handles():
    _flush("[gpu] batched boundaries vs single handles")
    states = [CASES[c]() for c in ("box", "mixed_inflow", "shock_reflection",
                                   "box_xwall_yper")]
    states.append(I.fourier_state(I.SEED_BASE + 6900, I.Grid(20, 20, 0.0, 1.0, 0.0, 1.0),
                                  I.GAMMA, 3))
    b = af.BatchSolver.for_states(states, precision=1, linearisation=1)
    b.run(1e9, 0.3, 5)
    for g, st in enumerate(states):
        s = af.Solver.for_state(st, precision=1, linearisation=1)
        s.run(1e9, 0.3, 5)
        ref = s.get_state()
        s.close()
        out = b.get_state(g)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], ref[k]), (g, k)
    b.close()


def test_inflow_arguments():
    _flush("[gpu] inflow argument checks")
    st = I.shock_reflection_state(24, 6)
    g = st.grid
    s = af.Solver(g.nx, g.ny, g.x0, g.x1, g.y0, g.y1, sides=g.side_kinds())
    s.set_state(st.avg, st.K, st.X, st.Y)
    with pytest.raises(af.AfError) as ei:  # no inflow state yet
        s.run(1e9, 0.3, 1)
    assert ei.value.code == af.AF_ERR_INVALID_ARG and "inflow" in str(ei.value)
    with pytest.raises(af.AfError):
        s.set_inflow(af.AF_SIDE_RIGHT, (1, 0, 0, 1))  # an outflow side
    with pytest.raises(af.AfError):
        s.set_inflow(af.AF_SIDE_LEFT, (0.0, 1, 0, 1))  # rho = 0
    with pytest.raises(af.AfError):
        s.set_inflow(4, (1, 0, 0, 1))
    s.set_inflow(af.AF_SIDE_LEFT, I.SRP_UP)
    with pytest.raises(af.AfError):  # the top side still has none
        s.step(1e-4)
    s.set_inflow(af.AF_SIDE_TOP, I.SRP_POST)
    t, n = s.run(1e9, 0.3, 3)
    assert n == 3
    out = s.get_state()
    e, _, _ = oracle.run(st, 1e9, 0.3, max_steps=3)
    assert e == 0
    _assert_close(out, st, 1e-12, "after set_inflow")
    # a changed inflow state applies from the next step on (the captured graphs are rebuilt)
    s.set_inflow(af.AF_SIDE_LEFT, (1.2, 2.9, 0.0, 0.8))
    s.run(1e9, 0.3, 2)
    out2 = s.get_state()
    st2 = I.State(I.Grid(g.nx, g.ny, g.x0, g.x1, g.y0, g.y1, sides=g.side_kinds(),
                         inflow=((1.2, 2.9, 0.0, 0.8), None, None, I.SRP_POST)),
                  st.gamma, st.avg, st.K, st.X, st.Y, st.t)
    e, _, _ = oracle.run(st2, 1e9, 0.3, max_steps=2)
    assert e == 0
    _assert_close(out2, st2, 1e-12, "changed inflow")
    s.close()
    # the kind must be known and periodic must pair
    with pytest.raises(af.AfError):
        af.Solver(8, 8, 0, 1, 0, 1, sides=(4, 1, 1, 1))
    with pytest.raises(af.AfError):
        af.Solver(8, 8, 0, 1, 0, 1, sides=(0, 2, 1, 1))


def _region_mean(out, grid, x0, x1, y0, y1):
    """Mean primitive cell average over the cells whose centres lie in the box."""
    xc, yc = grid.cell_centres()
    m = (xc > x0) & (xc < x1) & (yc > y0) & (yc < y1)
    Q = out["avg"][:, m]
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    p = (I.GAMMA - 1) * (Q[3] - 0.5 * rho * (u * u + v * v))
    return np.array([rho.mean(), u.mean(), v.mean(), p.mean()]), int(m.sum())


@pytest.mark.parametrize("nx,ny,mode", [(120, 30, 1), (240, 60, 1), (240, 60, 0)])
def test_shock_reflection_reaches_exact_states(nx, ny, mode):
    """The shock-reflection problem (inflow left and top, wall below, outflow right) to t = 6
    without limiter: upstream of the incident shock the inflow state, between the shocks the
    given post-shock state, and between the reflected shock and the wall the state that turns
    the flow back parallel to the wall (exact oblique-shock relations), sampled in boxes away
    from the shocks."""
    _flush(f"[gpu] shock reflection {nx}x{ny} mode={mode} to t=6")
    st = I.shock_reflection_state(nx, ny)
    s = af.Solver.for_state(st, precision=0, linearisation=mode)
    t, n = s.run(6.0, 0.3)
    out = s.get_state()
    s.close()
    assert t == 6.0
    up = np.array(I.SRP_UP)
    post = np.array(I.SRP_POST)
    theta = -math.atan2(post[2], post[1])
    beta = ES.weak_shock_angle(post, theta)
    refl = ES.turned_state(post, beta, +1)
    # incident shock y = 1 - x tan 29deg meets the wall at x_r; reflected shock
    # y = (x - x_r) tan(beta - theta)
    xr = 1.0 / math.tan(math.radians(29.0))
    wr = math.tan(beta - theta)
    def shock_y(x):  # the lower shock: incident before x_r, reflected after
        return 1 - x * math.tan(math.radians(29.0)) if x < xr else (x - xr) * wr

    g = st.grid
    # the sampling boxes keep 0.1 from the shocks
    assert shock_y(0.2) > 0.3 + 0.1 and shock_y(0.9) > 0.3 + 0.1
    r1, c1 = _region_mean(out, g, 0.2, 0.9, 0.05, 0.3)
    assert shock_y(1.8) < 0.75 - 0.1 and shock_y(2.6) < 0.75 - 0.1
    r2, c2 = _region_mean(out, g, 1.8, 2.6, 0.75, 0.95)
    assert shock_y(3.0) > 0.3 + 0.1
    r3, c3 = _region_mean(out, g, 3.0, 3.9, 0.05, 0.3)
    _flush(f"  region 1 {r1} ({c1} cells)\n  region 2 {r2} ({c2})\n  region 3 {r3} ({c3}) "
           f"exact {refl}")
    for r, ex, lab in ((r1, up, "upstream"), (r2, post, "between shocks"),
                       (r3, refl, "reflected")):
        err = np.abs(r - ex)
        assert err[0] < 0.01 * ex[0] and err[3] < 0.01 * ex[3], (lab, r, ex)
        assert err[1] < 0.01 * abs(ex[1]) and err[2] < 0.01 * max(abs(ex[1]), 1.0), \
            (lab, r, ex)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_shock_reflection_benchmark_grid_matches_oracle(prec, tol):
    """The 240 x 60 shock-reflection grid the benchmark's extra workloads time (averaged
    linearisation, no limiter): 6 steps against the oracle, every DOF."""
    _flush(f"[gpu] shock reflection 240x60 vs oracle prec={prec}")
    st = I.shock_reflection_state(240, 60)
    s = af.Solver.for_state(st, precision=prec, linearisation=af.AF_LIN_AVG)
    t, n = s.run(1e9, 0.3, 6)
    out = s.get_state()
    s.close()
    e, n2, _ = oracle.run(st, 1e9, 0.3, max_steps=6, mode=oracle.MODE_AVG)
    assert e == 0 and n == n2 == 6
    _assert_close(out, st, tol, f"240x60 prec {prec}")
