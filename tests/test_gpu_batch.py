"""Batched grids (af_create_batch): many independent grids advanced with one launch of each
kernel per step.

The batched kernels run the same per-DOF arithmetic as the single-grid kernels (only the
mapping of workgroups to tiles and rows differs, and the wave-speed maximum is order
independent), so a batch must reproduce separate single-grid handles bit for bit, each grid
with its own time step.  Against the FP64 oracle the tolerance is the single-grid one.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_states():
    """Uneven grids: ragged tile counts, an outflow grid, a non-square domain, a tiny grid."""
    out = [I.fourier_state(11, I.Grid(37, 29, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
           I.fourier_state(12, I.Grid(16, 16, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
           I.fourier_state(13, I.Grid(9, 11, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
           I.shu_vortex(40, n_gl=3),
           I.radial_state(24, n_gl=3, noise=0.0)]
    g = out[4].grid
    assert g.bc_x == I.BC_OUTFLOW
    return out


def _singles(states, steps, **kw):
    res = []
    for st in states:
        s = af.Solver.for_state(st, **kw)
        t, n = s.run(1e9, 0.3, steps)
        res.append((s.get_state(), n, s.counters()))
        s.close()
    return res


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode,limiter", [(0, False), (1, True)])
def test_batch_equals_single_handles(prec, mode, limiter):
    _flush(f"[gpu] batch vs single handles prec={prec} mode={mode} limiter={limiter}")
    states = _mixed_states()
    kw = dict(precision=prec, linearisation=mode, limiter=limiter)
    ref = _singles(states, 7, **kw)
    b = af.BatchSolver.for_states(states, **kw)
    assert len(b) == len(states)
    t, n = b.run(1e9, 0.3, 7)
    assert n == 7
    for g, (out_s, n_s, _) in enumerate(ref):
        out_b = b.get_state(g)
        tg, ng = b.grid_info(g)
        assert ng == n_s == 7
        assert tg == out_s["t"]
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out_b[k], out_s[k]), (g, k)
    cnt = b.counters()
    tot = sum(c for (_, _, c) in ref)
    assert list(cnt[:4]) == list(tot[:4])
    assert b.dof_count() == sum(st.grid.dof_count() for st in states)
    b.close()


def test_batch_matches_oracle_fp64():
    _flush("[gpu] batch vs oracle, 3 grids x 4 steps")
    states = _mixed_states()[:3]
    b = af.BatchSolver.for_states(states)
    b.run(1e9, 0.3, 4)
    for g, st in enumerate(states):
        e, n, _ = oracle.run(st, 1e9, 0.3, max_steps=4)
        assert e == 0 and n == 4
        out = b.get_state(g)
        scale = max(float(np.abs(st.avg).max()), float(np.abs(st.K).max()))
        for k in ("avg", "K", "X", "Y"):
            assert np.abs(out[k] - getattr(st, k)).max() < 1e-12 * scale, (g, k)
    b.close()


def test_batch_each_grid_lands_on_t_end():
    """Own time step per grid: a coarse and a fine grid reach the same t_end with different
    step counts, each exactly, as separate handles do."""
    _flush("[gpu] batch per-grid t_end")
    states = [I.fourier_state(21, I.Grid(12, 12, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
              I.fourier_state(22, I.Grid(48, 48, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)]
    t_end = 0.05
    b = af.BatchSolver.for_states(states)
    t, n = b.run(t_end, 0.3)
    info = [b.grid_info(g) for g in range(2)]
    assert info[0][0] == t_end and info[1][0] == t_end
    assert info[1][1] > info[0][1]
    for g, st in enumerate(states):
        s = af.Solver.for_state(st)
        ts, ns = s.run(t_end, 0.3)
        assert ts == t_end and ns == info[g][1]
        ref = s.get_state()
        out = b.get_state(g)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], ref[k])
        s.close()
    assert t == t_end and n == info[1][1]
    b.close()


def test_batch_step_error_stays_in_its_grid():
    """af_step with one dt for all grids: the fine grid violates its CFL bound and keeps its
    state; the coarse grid advances; the error names the failing grid."""
    _flush("[gpu] batch step error isolation")
    coarse = I.fourier_state(31, I.Grid(8, 8, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)
    fine = I.fourier_state(32, I.Grid(64, 64, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)
    b = af.BatchSolver.for_states([coarse, fine])
    dt = 0.3 / 8 / 1.6  # within the coarse grid's bound, far beyond the fine grid's
    with pytest.raises(af.AfError) as ei:
        b.step(dt)
    assert ei.value.code == af.AF_ERR_CFL and "grid 1" in str(ei.value)
    out_f = b.get_state(1)
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(out_f[k], getattr(fine, k))
    assert b.grid_info(1) == (0.0, 0)
    tc, nc = b.grid_info(0)
    assert nc == 1 and tc == dt
    s = af.Solver.for_state(coarse)
    s.step(dt)
    ref = s.get_state()
    out_c = b.get_state(0)
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(out_c[k], ref[k])
    s.close()
    b.close()


def test_batch_bad_arguments():
    import ctypes as ct
    states = _mixed_states()[:2]
    b = af.BatchSolver.for_states(states)
    P = lambda a: np.ascontiguousarray(a).ctypes.data_as(ct.POINTER(ct.c_double))
    st = states[0]
    # grid index out of range: refused by the library before any copy
    assert b.L.af_set_state_grid(b.h, 2, P(st.avg), P(st.K), P(st.X), P(st.Y), 0.0) == \
        af.AF_ERR_INVALID_ARG
    out = np.zeros(st.avg.shape)
    assert b.L.af_get_state_grid(b.h, -1, P(out), None, None, None, None) == \
        af.AF_ERR_INVALID_ARG
    # the single-grid calls refuse a handle with several grids
    assert b.L.af_get_state(b.h, P(out), None, None, None, None) == af.AF_ERR_INVALID_ARG
    # shapes are checked by the binding
    with pytest.raises(ValueError):
        b.set_state(0, states[1].avg, states[1].K, states[1].X, states[1].Y)
    b.close()
    with pytest.raises(af.AfError):
        af.BatchSolver([])


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_workload_full_size_sampled(prec):
    """The batched workload at its full size (256 periodic grids, N ~ U{64..512}), in the launch
    configuration the benchmark times: 3 steps, then the three smallest grids are compared bit
    for bit with single-grid handles and the smallest with the oracle."""
    _flush(f"[gpu] batched workload 256 grids, prec={prec}")
    sizes = I.batched_sizes()
    states = I.batched_states(n_gl=2, sizes=sizes)
    b = af.BatchSolver.for_states(states, precision=prec)
    t, n = b.run(1e9, 0.3, 3)
    assert n == 3
    small = list(np.argsort(sizes, kind="stable")[:3])
    for g in small:
        s = af.Solver.for_state(states[g], precision=prec)
        s.run(1e9, 0.3, 3)
        ref = s.get_state()
        out = b.get_state(int(g))
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], ref[k]), (g, k)
        s.close()
    g0 = int(small[0])
    st = states[g0]
    e, n2, _ = oracle.run(st, 1e9, 0.3, max_steps=3)
    assert e == 0 and n2 == 3
    out = b.get_state(g0)
    tol = 1e-12 if prec == 0 else 1e-5
    scale = max(float(np.abs(st.avg).max()), float(np.abs(st.K).max()))
    for k in ("avg", "K", "X", "Y"):
        assert np.abs(out[k] - getattr(st, k)).max() < tol * scale, k
    b.close()


def test_batch_schedules_give_identical_results():
    """Every tile order and update workgroup size, and the autotuned choice, compute the same
    bits (the schedule only maps workgroups to tiles and rows)."""
    _flush("[gpu] batch schedules and autotuner")
    states = _mixed_states()
    ref = None
    for order in (af.AF_ORDER_XCD, af.AF_ORDER_LINEAR, af.AF_ORDER_GRIDS):
        for threads in (64, 128, 256):
            b = af.BatchSolver.for_states(states, precision=1)
            b.set_option(af.AF_OPT_TILE_ORDER, order)
            b.set_option(af.AF_OPT_UPDATE_THREADS, threads)
            assert b.get_option(af.AF_OPT_TILE_ORDER) == order
            assert b.get_option(af.AF_OPT_UPDATE_THREADS) == threads
            b.run(1e9, 0.3, 20)
            out = [b.get_state(g) for g in range(len(states))]
            b.close()
            if ref is None:
                ref = out
            for g in range(len(states)):
                for k in ("avg", "K", "X", "Y"):
                    assert np.array_equal(out[g][k], ref[g][k]), (order, threads, g, k)
    b = af.BatchSolver.for_states(states, precision=1)
    b.set_option(af.AF_OPT_AUTOTUNE, 1)
    t, n = b.run(1e9, 0.3, 20)
    assert n == 20
    assert b.get_option(af.AF_OPT_TILE_ORDER) in (0, 1, 2)
    assert b.get_option(af.AF_OPT_UPDATE_THREADS) in (64, 128, 256)
    assert b.get_option(af.AF_OPT_AUTOTUNE) == 0  # tuned once
    for g in range(len(states)):
        out = b.get_state(g)
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(out[k], ref[g][k]), ("autotuned", g, k)
    with pytest.raises(af.AfError):
        b.set_option(af.AF_OPT_UPDATE_THREADS, 96)
    with pytest.raises(af.AfError):
        b.set_option(af.AF_OPT_TILE_ORDER, 3)
    b.close()
    s = af.Solver.for_state(states[0])
    with pytest.raises(af.AfError):
        s.set_option(af.AF_OPT_TILE_ORDER, 0)
    s.close()



def test_timing_counts_only_steps_that_ran():
    """With AF_OPT_TIMING the batched run still enqueues whole chunks of steps; the launches
    after every grid has reached its step limit or t_end return at once and must not enter the
    mean kernel times.  The count that af_get_timing reports is the number of steps taken,
    for single and batched handles alike, and a real step is not shorter than a third of the
    single-grid step on the same grid (a mean over no-op launches would be)."""
    _flush("[gpu] timing counts only executed steps")
    st = I.fourier_state(1, I.Grid(512, 512, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 2)
    s = af.Solver.for_state(st, precision=1)
    s.set_option(af.AF_OPT_TIMING, 1)
    t, n = s.run(1e9, 0.3, 3)
    mp_s, mu_s, n_s = s.timing()
    s.close()
    assert n == 3 and n_s == 3
    b = af.BatchSolver.for_states([st], precision=1)
    b.set_option(af.AF_OPT_TIMING, 1)
    t, n = b.run(1e9, 0.3, 3)  # one chunk of 16 launches, 13 of them no-ops
    mp_b, mu_b, n_b = b.timing()
    b.close()
    _flush(f"  single {mp_s / n_s:.4f} ms, batched {mp_b / n_b:.4f} ms per point kernel")
    assert n == 3 and n_b == 3
    assert mp_b / n_b > (mp_s / n_s) / 3.0


def _batch_sweep_cases(n=20, seed=I.SEED_BASE + 39400):
    PER, OUT, WALL, INFLOW = I.BC_PERIODIC, I.BC_OUTFLOW, I.BC_WALL, I.BC_INFLOW
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ng = int(rng.integers(2, 7))
        states = []
        for g in range(ng):
            nx, ny = int(rng.integers(3, 70)), int(rng.integers(3, 70))
            sides = []
            for axis in range(2):
                if rng.random() < 0.4:
                    sides += [PER, PER]
                else:
                    sides += [int(rng.choice([OUT, WALL, INFLOW])) for _ in range(2)]
            inflow = tuple((float(rng.uniform(0.9, 1.1)), float(rng.uniform(-0.2, 0.2)),
                            float(rng.uniform(-0.2, 0.2)), float(rng.uniform(0.9, 1.1)))
                           if s == INFLOW else None for s in sides)
            dx = float(rng.uniform(0.02, 0.1))
            grid = I.Grid(nx, ny, 0.0, nx * dx, 0.0, ny * dx * float(rng.uniform(0.5, 2.0)),
                          sides=tuple(sides), inflow=inflow if INFLOW in sides else None)
            states.append(I.fourier_state(int(rng.integers(1, 10 ** 6)), grid, I.GAMMA, 3))
        opts = dict(precision=int(rng.integers(0, 2)), linearisation=int(rng.integers(0, 3)),
                    limiter=bool(rng.random() < 0.5), transonic=bool(rng.random() < 0.3),
                    shock_limiter=bool(rng.random() < 0.3))
        out.append((states, opts, int(rng.integers(0, 2))))
    return out


BATCH_SWEEP = _batch_sweep_cases()


@pytest.mark.parametrize("k", range(len(BATCH_SWEEP)))
def test_batch_sweep_equals_single_handles(k):
    """Random batches: 2 to 6 grids of 3 to 69 cells per side, every kind of side (inflow
    states per grid), random options (precision, linearisation, limiter, Algorithm 2, the
    Sec. 3.4 blend) and either step kernel: 5 steps of the batch equal separate single-grid
    handles bit for bit, each grid with its own time step."""
    states, opts, kernel = BATCH_SWEEP[k]
    _flush(f"[gpu] batch sweep case {k}: {len(states)} grids, {opts}, step kernel {kernel}")
    b = af.BatchSolver.for_states(states, **opts)
    b.set_option(af.AF_OPT_STEP_KERNEL, kernel)
    t, n = b.run(1e9, 0.3, 5)
    assert n == 5
    outs = [b.get_state(g) for g in range(len(states))]
    b.close()
    for g, st in enumerate(states):
        s = af.Solver.for_state(st, **opts)
        s.run(1e9, 0.3, 5)
        ref = s.get_state()
        s.close()
        for key in ("avg", "K", "X", "Y"):
            assert np.array_equal(outs[g][key], ref[key]), (g, key)
