"""The persistent step kernel of batched handles (AF_OPT_STEP_KERNEL = AF_STEP_PERSISTENT): the
whole step of every grid in one launch, with device-side queues and grid-wide barriers between
the phases.

It runs the same per-DOF and per-cell arithmetic as the separate kernels; only the assignment
of tiles and update chunks to workgroups differs, and every reduction across workgroups is
order independent (maxima of wave speeds, counter sums).  So it must reproduce the separate
kernels bit for bit, in every option set, over several steps (which checks that the kernel
leaves its queues and counters ready for the next launch), through graph replays and eager
launches alike.
"""
import sys

import numpy as np
import pytest

from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_states():
    """Uneven grids: ragged tile counts, an outflow grid, a tiny grid, odd widths."""
    return [I.fourier_state(11, I.Grid(37, 29, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
            I.fourier_state(12, I.Grid(16, 16, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
            I.fourier_state(13, I.Grid(9, 11, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
            I.shu_vortex(40, n_gl=3),
            I.radial_state(24, n_gl=3, noise=0.0)]


def _run(states, kernel, steps, timing=False, order=None, **kw):
    b = af.BatchSolver.for_states(states, **kw)
    b.set_option(af.AF_OPT_STEP_KERNEL, kernel)
    assert b.get_option(af.AF_OPT_STEP_KERNEL) == kernel
    if order is not None:
        b.set_option(af.AF_OPT_TILE_ORDER, order)
    if timing:
        b.set_option(af.AF_OPT_TIMING, 1)  # eager launches
    t, n = b.run(1e9, 0.3, steps)
    out = [b.get_state(g) for g in range(len(states))]
    info = [b.grid_info(g) for g in range(len(states))]
    cnt = b.counters()
    b.close()
    return t, n, out, info, cnt


def _same(a, b, label):
    for g in range(len(a)):
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(a[g][k], b[g][k]), (label, g, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("opts", [dict(linearisation=0), dict(linearisation=1, limiter=True),
                                  dict(linearisation=2, correction=False)],
                         ids=["af3", "avg-limiter", "simple"])
def test_persistent_equals_split(prec, opts):
    _flush(f"[gpu] persistent vs split prec={prec} {opts}")
    states = _mixed_states()
    ref = _run(states, af.AF_STEP_SPLIT, 11, precision=prec, **opts)
    out = _run(states, af.AF_STEP_PERSISTENT, 11, precision=prec, **opts)
    assert out[0] == ref[0] and out[1] == ref[1] == 11
    assert out[3] == ref[3]
    assert list(out[4]) == list(ref[4])
    _same(out[2], ref[2], "graph")
    # eager launches (timing on) and a different tile order: the same bits
    eager = _run(states, af.AF_STEP_PERSISTENT, 11, timing=True, order=af.AF_ORDER_GRIDS,
                 precision=prec, **opts)
    assert eager[3] == ref[3]
    _same(eager[2], ref[2], "eager")


def _riemann(grid):
    """Four constant states meeting at the domain's centre (transonic shocks, jumps)."""
    Q = (np.array([1.0, 1.3, 1.3, 0.7]), np.array([1.8, -0.1, 1.3, 2.0]),
         np.array([1.8, 1.3, -0.1, 2.0]), np.array([2.5, -0.2, -0.2, 3.0]))
    xs, ys = 0.5 * (grid.x0 + grid.x1), 0.5 * (grid.y0 + grid.y1)

    def prim(x, y, sites):
        W = np.zeros((4,) + np.shape(x))
        for q, (r, t) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
            wx = (x > xs) * 1.0 if r else (x < xs) * 1.0
            wy = (y > ys) * 1.0 if t else (y < ys) * 1.0
            if sites:
                wx = wx + 0.5 * (x == xs)
                wy = wy + 0.5 * (y == ys)
            W += Q[q].reshape((4,) + (1,) * np.ndim(x)) * (wx * wy)[None]
        return W

    avg = I.cell_average(lambda x, y: prim(x, y, False), grid, I.GAMMA, 3)
    return I.State(grid, I.GAMMA, avg, prim(*grid.k_sites(), True),
                   prim(*grid.x_sites(), True), prim(*grid.y_sites(), True))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("limiter", [False, True])
def test_persistent_indicators_equal_split(prec, limiter):
    """With Algorithm 2 and the Sec. 3.4 blend: the persistent kernel adds a first phase (the
    padded primitive averages) and the indicator variant of the tiles."""
    _flush(f"[gpu] persistent vs split, indicators, prec={prec} limiter={limiter}")
    # outflow grids run these data without the limiter (checked with the oracle); the periodic
    # grid needs Algorithm 3 once its shocks wrap around
    states = [_riemann(I.Grid(41, 9, 0.0, 2.0, 0.0, 0.5, sides=(I.BC_OUTFLOW,) * 4)),
              _riemann(I.Grid(24, 20, 0.0, 1.0, 0.0, 1.0, sides=(I.BC_OUTFLOW,) * 4))]
    if limiter:
        states.append(_riemann(I.Grid(30, 22, 0.0, 1.0, 0.0, 0.8)))
    kw = dict(precision=prec, linearisation=1, limiter=limiter, transonic=True,
              shock_limiter=True)
    ref = _run(states, af.AF_STEP_SPLIT, 9, **kw)
    out = _run(states, af.AF_STEP_PERSISTENT, 9, **kw)
    assert out[1] == ref[1] == 9 and out[3] == ref[3]
    assert list(out[4]) == list(ref[4])
    assert int(ref[4][af.AF_CNT_TSW]) > 0
    _same(out[2], ref[2], "indicators")


def test_persistent_host_dt_and_error_isolation():
    """af_step with one dt for all grids: the fine grid violates its CFL bound and keeps its
    state, the coarse grid advances, as with the separate kernels."""
    _flush("[gpu] persistent af_step, error in one grid")
    coarse = I.fourier_state(31, I.Grid(8, 8, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)
    fine = I.fourier_state(32, I.Grid(64, 64, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)
    res = {}
    for kernel in (af.AF_STEP_SPLIT, af.AF_STEP_PERSISTENT):
        b = af.BatchSolver.for_states([coarse, fine])
        b.set_option(af.AF_OPT_STEP_KERNEL, kernel)
        dt = 0.3 / 8 / 1.6
        with pytest.raises(af.AfError) as ei:
            b.step(dt)
        assert ei.value.code == af.AF_ERR_CFL and "grid 1" in str(ei.value)
        assert b.grid_info(1) == (0.0, 0) and b.grid_info(0) == (dt, 1)
        out_f = b.get_state(1)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out_f[k], getattr(fine, k))
        # a good step afterwards: both grids advance
        b.step(dt / 8)
        res[kernel] = [b.get_state(g) for g in range(2)]
        assert b.grid_info(0)[1] == 2 and b.grid_info(1)[1] == 1
        b.close()
    _same(res[af.AF_STEP_PERSISTENT], res[af.AF_STEP_SPLIT], "af_step")


@pytest.mark.parametrize("prec", [0, 1])
def test_persistent_runs_that_stop_inside_a_chunk(prec):
    """Grids that reach t_end at different steps, so that the last launches of the graph chunk
    find no grid that can step (the persistent kernel then leaves at once); then one af_step
    with a host dt past t_end, and a run cut by its step limit (launched without a graph).
    Every state, time and step count equals the separate kernels'."""
    _flush(f"[gpu] persistent runs stopping inside a chunk, prec={prec}")
    states = _mixed_states()
    res = {}
    for kernel in (af.AF_STEP_SPLIT, af.AF_STEP_PERSISTENT):
        b = af.BatchSolver.for_states(states, precision=prec)
        b.set_option(af.AF_OPT_STEP_KERNEL, kernel)
        t, n = b.run(0.05, 0.3)
        assert t == 0.05 and 1 < n < 16  # the chunk ends with launches that step no grid
        steps = [b.grid_info(g)[1] for g in range(len(states))]
        assert len(set(steps)) > 1
        b.step(1e-3)
        t2, n2 = b.run(0.2, 0.3, 5)
        assert n2 == 5
        res[kernel] = ([b.get_state(g) for g in range(len(states))],
                       [b.grid_info(g) for g in range(len(states))], b.counters())
        b.close()
    _same(res[af.AF_STEP_PERSISTENT][0], res[af.AF_STEP_SPLIT][0], "stop inside a chunk")
    assert res[af.AF_STEP_PERSISTENT][1] == res[af.AF_STEP_SPLIT][1]
    assert np.array_equal(res[af.AF_STEP_PERSISTENT][2], res[af.AF_STEP_SPLIT][2])


@pytest.mark.parametrize("prec", [1, 0])
def test_persistent_full_size_workload(prec):
    """The batched workload at full size (256 periodic grids, N ~ U{64..512}): more tiles than
    resident workgroups, so every workgroup takes many items.  Three steps equal the separate
    kernels' on every grid."""
    _flush(f"[gpu] persistent, 256-grid workload, prec={prec}")
    states = I.batched_states(n_gl=2)
    ref = _run(states, af.AF_STEP_SPLIT, 3, precision=prec)
    out = _run(states, af.AF_STEP_PERSISTENT, 3, precision=prec)
    assert out[1] == ref[1] == 3 and out[3] == ref[3]
    _same(out[2], ref[2], "workload")


@pytest.mark.parametrize("prec", [1, 0])
def test_persistent_full_size_workload_with_indicators(prec):
    """The same workload with Algorithm 2, the Sec. 3.4 blend and Algorithm 3 on: the
    persistent kernel's indicator variant, with its padded-average phase over every row of the
    256 grids, equals the separate kernels on every grid, counters included."""
    _flush(f"[gpu] persistent, 256-grid workload with indicators and limiter, prec={prec}")
    states = I.batched_states(n_gl=2)
    kw = dict(precision=prec, linearisation=1, limiter=True, transonic=True,
              shock_limiter=True)
    ref = _run(states, af.AF_STEP_SPLIT, 3, **kw)
    out = _run(states, af.AF_STEP_PERSISTENT, 3, **kw)
    assert out[1] == ref[1] == 3 and out[3] == ref[3]
    assert list(out[4]) == list(ref[4])
    _same(out[2], ref[2], "workload with indicators")


def test_persistent_option_and_autotuner():
    _flush("[gpu] persistent option, autotuner")
    states = _mixed_states()
    b = af.BatchSolver.for_states(states, precision=1)
    assert b.get_option(af.AF_OPT_STEP_KERNEL) == af.AF_STEP_SPLIT
    with pytest.raises(af.AfError):
        b.set_option(af.AF_OPT_STEP_KERNEL, 2)
    b.set_option(af.AF_OPT_AUTOTUNE, 1)
    t, n = b.run(1e9, 0.3, 12)
    assert n == 12
    assert b.get_option(af.AF_OPT_STEP_KERNEL) in (af.AF_STEP_SPLIT, af.AF_STEP_PERSISTENT)
    out = [b.get_state(g) for g in range(len(states))]
    b.close()
    ref = _run(states, af.AF_STEP_SPLIT, 12, precision=1)
    _same(out, ref[2], "autotuned")
    s = af.Solver.for_state(states[0])
    with pytest.raises(af.AfError):
        s.set_option(af.AF_OPT_STEP_KERNEL, af.AF_STEP_PERSISTENT)
    s.close()


def test_persistent_barrier_timeout_keeps_the_state():
    """The persistent kernel's barrier waits are bounded.  With the limit set to 0 from the host
    (AF_OPT_SYNC_TIMEOUT_US) the workgroups that reach a barrier first stop waiting at once: the
    step is abandoned with AF_ERR_DEVICE, every kernel still ends, and each grid keeps its t_n
    state (the step writes only the other buffer).  With the default limit restored the next
    steps equal the separate kernels' bit for bit.  Limiter and indicators off: their phases
    read lists that an abandoned barrier would leave half written."""
    _flush("[gpu] persistent barrier timeout")
    states = _mixed_states()
    dt = 2e-4
    ref = af.BatchSolver.for_states(states, precision=1)
    for _ in range(3):
        ref.step(dt)
    want = [ref.get_state(g) for g in range(len(states))]
    ref.close()
    b = af.BatchSolver.for_states(states, precision=1)
    b.set_option(af.AF_OPT_STEP_KERNEL, af.AF_STEP_PERSISTENT)
    assert b.get_option(af.AF_OPT_SYNC_TIMEOUT_US) == 2000000
    b.set_option(af.AF_OPT_SYNC_TIMEOUT_US, 0)
    with pytest.raises(af.AfError) as ei:
        b.step(dt)
    assert ei.value.code == af.AF_ERR_DEVICE and "barrier" in str(ei.value)
    for g, st in enumerate(states):
        assert b.grid_info(g) == (0.0, 0)
        out = b.get_state(g)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], getattr(st, k)), (g, k)
    b.set_option(af.AF_OPT_SYNC_TIMEOUT_US, 2000000)
    for _ in range(3):
        b.step(dt)
    _same([b.get_state(g) for g in range(len(states))], want, "after timeout")
    with pytest.raises(af.AfError):
        b.set_option(af.AF_OPT_SYNC_TIMEOUT_US, -1)
    b.close()
    s = af.Solver.for_state(states[0])
    with pytest.raises(af.AfError):
        s.set_option(af.AF_OPT_SYNC_TIMEOUT_US, 10)
    s.close()
