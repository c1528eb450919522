"""af_step_noalloc (the entry point that allocates nothing) against af_step on a handle, through
the C ABI: two calls in a row on one GPU, the second on a smaller grid, each compared with the
handle path (same kernels and arithmetic: bit for bit, and the FP64 parity bar of 1e-12 in any
case), counters included."""
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


def _pitches(g):
    return (g.nx + 31) // 32 * 32, (g.nkx + 63) // 64 * 64


def _to_device(st):
    """The state in the library's device layout (torch tensors on cuda:0)."""
    g = st.grid
    pa, pp = _pitches(g)
    dev = {}
    a = np.zeros((4, g.ny, pa))
    a[:, :, :g.nx] = st.avg
    dev["avg"] = torch.from_numpy(a).cuda()
    for k in ("K", "X", "Y"):
        b = np.zeros((4, g.nky, pp))
        src = getattr(st, k)
        b[:, :src.shape[1], :src.shape[2]] = src
        dev[k] = torch.from_numpy(b).cuda()
    return dev, pa, pp


def _from_device(dev, st):
    out = {"avg": dev["avg"].cpu().numpy()[:, :st.grid.ny, :st.grid.nx]}
    for k in ("K", "X", "Y"):
        shp = getattr(st, k).shape
        out[k] = dev[k].cpu().numpy()[:, :shp[1], :shp[2]]
    return out


def _one(st, dt, prec, mode, limiter):
    g = st.grid
    sides = g.side_kinds()
    h = af.Solver.for_state(st, precision=prec, linearisation=mode, limiter=limiter)
    h.step(dt)
    ref = h.get_state()
    ref_cnt = h.counters()
    h.close()
    ins, pa, pp = _to_device(st)
    outs = {k: torch.full_like(v, float("nan")) for k, v in ins.items()}
    torch.cuda.synchronize()
    cnt = af.step_noalloc((g.nx, g.ny, g.x0, g.x1, g.y0, g.y1), st.gamma, sides,
                          [ins[k].data_ptr() for k in ("avg", "K", "X", "Y")],
                          [outs[k].data_ptr() for k in ("avg", "K", "X", "Y")], pa, pp, dt,
                          precision=prec, linearisation=mode, limiter=limiter,
                          stream=torch.cuda.current_stream().cuda_stream)
    got = _from_device(outs, st)
    for k in ("avg", "K", "X", "Y"):
        d = float(np.abs(got[k] - ref[k]).max())
        assert d <= 1e-12 * max(1.0, float(np.abs(ref[k]).max())), (k, d)
        assert np.array_equal(got[k], ref[k]), k
    assert list(cnt[:4]) == list(ref_cnt[:4]) and cnt[4] == 1
    return got


def test_noalloc_matches_handle_two_calls():
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    _flush("[gpu] af_step_noalloc: 64x48 periodic, FP64, Algorithm 1")
    g1 = I.Grid(64, 48, 0.0, 1.0, 0.0, 0.75)
    st1 = I.fourier_state(31, g1, I.GAMMA, 3)
    _one(st1, 0.25 * g1.dx, af.AF_PREC_FP64, af.AF_LIN_AF3, False)
    _flush("[gpu] af_step_noalloc: 19x13 outflow/wall, FP32, averaged linearisation, limiter")
    g2 = I.Grid(19, 13, -1.0, 1.0, -0.5, 0.8, sides=(1, 1, 2, 2))
    st2 = I.state_from_field(I.fourier_field(7), g2, I.GAMMA, 3)
    _one(st2, 0.1 * g2.dx, af.AF_PREC_FP32, af.AF_LIN_AVG, True)
