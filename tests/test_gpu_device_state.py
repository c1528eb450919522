"""State in device memory (af_set_state_device / af_get_state_device): the device-to-device path
gives the same bits as the host path, on single-grid and batched handles, and refuses a
non-admissible average found on the device."""
import sys

import numpy as np
import pytest

from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")
torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tensors(st):
    return [torch.from_numpy(np.ascontiguousarray(getattr(st, k))).to("cuda")
            for k in ("avg", "K", "X", "Y")]


def _empty_like(st):
    return [torch.empty(getattr(st, k).shape, dtype=torch.float64, device="cuda")
            for k in ("avg", "K", "X", "Y")]


def test_device_state_equals_host_state_single():
    _flush("[gpu] device state, single grid")
    st = I.fourier_state(I.SEED_BASE + 7200, I.Grid(37, 21, 0.0, 1.0, 0.0, 0.6), I.GAMMA, 3)
    a = af.Solver.for_state(st)
    a.run(1e9, 0.3, 4)
    ref = a.get_state()
    a.close()
    g = st.grid
    b = af.Solver(g.nx, g.ny, g.x0, g.x1, g.y0, g.y1)
    b.set_state_device(0, *_tensors(st), t=st.t)
    b.run(1e9, 0.3, 4)
    out = _empty_like(st)
    t = b.get_state_device(0, *out)
    b.close()
    assert t == ref["t"]
    for k, o in zip(("avg", "K", "X", "Y"), out):
        assert np.array_equal(o.cpu().numpy(), ref[k]), k


def test_device_state_batched_and_errors():
    _flush("[gpu] device state, batched grids and errors")
    states = [I.fourier_state(I.SEED_BASE + 7300, I.Grid(20, 20, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3),
              I.box_state(13, ny=9)]
    ref = af.BatchSolver.for_states(states)
    ref.run(1e9, 0.3, 3)
    b = af.BatchSolver([(st.grid.nx, st.grid.ny, st.grid.x0, st.grid.x1, st.grid.y0,
                         st.grid.y1, st.grid.side_kinds()) for st in states])
    for g, st in enumerate(states):
        b.set_state_device(g, *_tensors(st))
    b.run(1e9, 0.3, 3)
    for g, st in enumerate(states):
        out = _empty_like(st)
        b.get_state_device(g, *out)
        r = ref.get_state(g)
        for k, o in zip(("avg", "K", "X", "Y"), out):
            assert np.array_equal(o.cpu().numpy(), r[k]), (g, k)
    # a non-admissible average on the device is refused, the state is kept
    bad = _tensors(states[0])
    bad[0][3, 4, 5] = -1.0
    with pytest.raises(af.AfError) as ei:
        b.set_state_device(0, *bad)
    assert ei.value.code == af.AF_ERR_NONPHYSICAL
    assert b.grid_info(0)[1] == 3
    with pytest.raises(ValueError):
        b.set_state_device(1, *_tensors(states[0]))  # shapes of grid 0 given for grid 1
    # no grid 2: refused by the library itself
    ts = _tensors(states[0])
    assert b.L.af_set_state_device(b.h, 2, *[x.data_ptr() for x in ts], 0.0) == \
        af.AF_ERR_INVALID_ARG
    ref.close()
    b.close()
