"""Domain totals of the conserved variables (af_get_totals): the device reduction equals the
sum of the averages the state copies back, is the same bits on every call, stays constant
over a periodic run (the conservative update, eq. 2dfvm, changes the totals only by rounding),
and is the same for a grid of a batch as for the same grid alone."""
import sys

import numpy as np
import pytest

from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _host_totals(out, grid):
    return out["avg"].reshape(4, -1).sum(axis=1) * grid.dx * grid.dy


@pytest.mark.parametrize("prec", [0, 1])
def test_totals_match_the_state_and_are_conserved(prec):
    _flush(f"[gpu] totals, periodic Fourier data, prec={prec}")
    st = I.fourier_state(5, I.Grid(67, 45, 0.0, 1.3, 0.0, 0.9), I.GAMMA, 3)
    s = af.Solver.for_state(st, precision=prec)
    t0 = s.totals()
    ref = _host_totals(s.get_state(), st.grid)
    assert np.allclose(t0, ref, rtol=1e-13, atol=1e-15)
    assert np.array_equal(s.totals(), t0)  # a fixed reduction order
    for _ in range(4):
        s.run(1e9, 0.3, 5)
        tk = s.totals()
        assert np.allclose(tk, _host_totals(s.get_state(), st.grid), rtol=1e-13, atol=1e-15)
        # periodic grid: every total is kept up to the rounding of the face sums
        assert np.abs(tk - t0).max() <= 1e-12 * np.abs(t0).max(), (tk, t0)
    with pytest.raises(af.AfError):
        s.totals(1)
    s.close()


def test_batch_totals_equal_single_grid_totals():
    _flush("[gpu] totals of a batch")
    states = [I.fourier_state(7, I.Grid(30, 21, 0.0, 1.0, 0.0, 0.7), I.GAMMA, 3),
              I.box_state(20, sides=(I.BC_WALL,) * 4),
              I.shu_vortex(40, n_gl=3)]
    b = af.BatchSolver.for_states(states, precision=1)
    b.run(1e9, 0.3, 6)
    for g, st in enumerate(states):
        s = af.Solver.for_state(st, precision=1)
        s.run(1e9, 0.3, 6)
        assert np.array_equal(b.totals(g), s.totals()), g
        s.close()
    with pytest.raises(af.AfError):
        b.totals(3)
    b.close()
