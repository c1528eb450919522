"""The paper's one-dimensional rarefaction tests (Sec. 3.2, transonic rarefaction; Sec. 3.2,
double rarefaction), run as quasi-1D problems on the GPU: a few cells in y, periodic in y,
outflow in x; the point values on the initial jump take the paper's middle states.

* Transonic rarefaction (left shock, right rarefaction through the sonic point), t = 0.4 on
  [-1.5, 0.5], Algorithm 1 without limiting: the GPU path equals the oracle; against the exact
  Riemann solution (tests/exact_riemann.py) the density converges (L1 halves from 100 to 200
  cells) and the fan has no expansion shock at the sonic point (no neighbour jump larger than
  a few times the exact profile's) -- the paper's observation that no entropy fix is needed.
  Algorithm 2 flags no corner of a rarefaction, so it leaves the run unchanged, bit for bit.
* Double rarefaction (Linde and Roe's data, t = 0.3 on [0, 1]): the two rarefactions just
  touch, and a vacuum opens at x = 1/2 (p* = 0).  Reading: with averages required to keep
  rho > 0 and p > 0 (R8), the unlimited method stops at t = 0.0055 with a non-admissible
  average next to the opening vacuum, on the GPU and in the oracle alike; the paper reports
  the unlimited run as stable.  With the positivity limiter (Algorithm 3) and the flux
  limiting of the averages (Sec. 3.5) the run reaches t = 0.3 with every average admissible,
  equals the oracle, and the density converges to the exact solution with its vacuum (L1
  halves from 128 to 256 cells).
"""
import sys

import numpy as np
import pytest

import oracle
import exact_riemann as ER
from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")

G = I.GAMMA
E4 = (np.array([0.1, -2.0, 0.0, 0.1]), np.array([0.55, -1.5, 0.0, 0.55]),
      np.array([1.0, -1.0, 0.0, 1.0]))
E5 = (np.array([7.0, -1.0, 0.0, 0.2]), np.array([7.0, 0.0, 0.0, 0.2]),
      np.array([7.0, 1.0, 0.0, 0.2]))


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(W, x0, x1, xs, n, ny=2):
    """Left state W[0] for x < xs, right state W[2] for x > xs, W[1] on the line x = xs."""
    WL, WM, WR = W
    grid = I.Grid(n, ny, x0, x1, 0.0, ny * (x1 - x0) / n,
                  sides=(I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_PERIODIC, I.BC_PERIODIC))

    def prim(x, y, sites):
        sh = (4,) + (1,) * np.ndim(x)
        out = (x < xs)[None] * WL.reshape(sh) + (x > xs)[None] * WR.reshape(sh)
        if sites:
            out = out + (x == xs)[None] * WM.reshape(sh)
        return out * 1.0

    avg = I.cell_average(lambda x, y: prim(x, y, False), grid, G, 4)
    return I.State(grid, G, avg, prim(*grid.k_sites(), True), prim(*grid.x_sites(), True),
                   prim(*grid.y_sites(), True))


def _gpu(st, t_end, prec, **kw):
    s = af.Solver.for_state(st, precision=prec, **kw)
    t, n = s.run(t_end, 0.3)
    out = s.get_state()
    cnt = s.counters()
    s.close()
    return t, n, out, cnt


def _l1_rho(avg, W, xs, t, x0, x1):
    n = avg.shape[2]
    ex = ER.cell_averages(W[0], W[2], xs, t, np.linspace(x0, x1, n + 1), G, sub=32)
    return float(np.abs(avg[0, 0, :] - ex[0]).sum() * (x1 - x0) / n), ex


def _close(out, ref, tol):
    scale = max(float(np.abs(ref.avg).max()), float(np.abs(ref.K).max()))
    for k in ("avg", "K", "X", "Y"):
        d = float(np.abs(out[k] - getattr(ref, k)).max())
        assert d <= tol * scale, (k, d, tol * scale)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_transonic_rarefaction(prec, tol):
    _flush(f"[gpu] transonic rarefaction, prec={prec}")
    errs = {}
    for n in (100, 200):
        st = _state(E4, -1.5, 0.5, 0.0, n)
        t, steps, out, cnt = _gpu(st, 0.4, prec)
        assert t == 0.4
        if n == 100:
            ref = _state(E4, -1.5, 0.5, 0.0, n)
            e, n_or, _ = oracle.run(ref, 0.4, 0.3)
            assert e == 0 and n_or == steps
            _close(out, ref, tol)
            # Algorithm 2: a rarefaction has no flagged corner, the run is the same
            t2, steps2, out2, cnt2 = _gpu(st, 0.4, prec, transonic=True)
            assert int(cnt2[af.AF_CNT_TSW]) == 0 and steps2 == steps
            for k in ("avg", "K", "X", "Y"):
                assert np.array_equal(out2[k], out[k]), k
        errs[n], ex = _l1_rho(out["avg"], E4, 0.0, 0.4, -1.5, 0.5)
        if n == 200:
            # the fan of the right rarefaction: no neighbour jump well above the exact ones
            x = -1.5 + (np.arange(n) + 0.5) * 2.0 / n
            ps, us = ER.star_state(E4[0], E4[2])
            cs = np.sqrt(G * ps / (E4[2][0] * (ps / E4[2][3]) ** (1 / G)))
            fan = (x > (us + cs) * 0.4 + 0.02) & (x < (E4[2][1] + np.sqrt(G)) * 0.4 - 0.02)
            assert fan.sum() > 20
            jump = np.abs(np.diff(out["avg"][0, 0, :]))[fan[:-1]]
            jump_ex = np.abs(np.diff(ex[0]))[fan[:-1]]
            assert jump.max() <= 3.0 * jump_ex.max(), (jump.max(), jump_ex.max())
    _flush(f"    L1(rho) vs exact: 100 cells {errs[100]:.3e}, 200 cells {errs[200]:.3e}")
    assert errs[200] < 3.5e-3 and errs[100] / errs[200] > 1.7


def test_double_rarefaction_unlimited_stops_at_the_vacuum():
    """The unlimited method: a non-admissible average at the opening vacuum, at the same time
    on the GPU (FP64) and in the oracle."""
    _flush("[gpu] double rarefaction, unlimited")
    st = _state(E5, 0.0, 1.0, 0.5, 128)
    ref = _state(E5, 0.0, 1.0, 0.5, 128)
    e, n_or, _ = oracle.run(ref, 0.3, 0.3)
    assert e == oracle.ERR_NONPHYSICAL and 0 < n_or < 10
    s = af.Solver.for_state(st, precision=0)
    with pytest.raises(af.AfError) as ei:
        s.run(0.3, 0.3)
    assert ei.value.code == af.AF_ERR_NONPHYSICAL
    out = s.get_state()
    s.close()
    assert abs(out["t"] - ref.t) <= 1e-14 * ref.t  # the same last good step (dt sums to rounding)
    _close(out, ref, 1e-12)


@pytest.mark.parametrize("prec", [0, 1])
def test_double_rarefaction_limited(prec):
    _flush(f"[gpu] double rarefaction with Algorithm 3 and flux limiting, prec={prec}")
    kw = dict(linearisation=1, limiter=True, flux_limiter=True)
    errs = {}
    for n in (128, 256):
        st = _state(E5, 0.0, 1.0, 0.5, n)
        t, steps, out, cnt = _gpu(st, 0.3, prec, **kw)
        assert t == 0.3
        assert out["avg"][0].min() > 0.0
        assert int(cnt[af.AF_CNT_FLUX]) > 0  # the flux limiting is what keeps the averages
        errs[n], _ = _l1_rho(out["avg"], E5, 0.5, 0.3, 0.0, 1.0)
        if n == 128 and prec == 0:
            ref = _state(E5, 0.0, 1.0, 0.5, n)
            e, n_or, cnt_or = oracle.run(ref, 0.3, 0.3, mode=1, limiter=True, flux_limiter=True)
            assert e == 0 and n_or == steps
            assert [int(cnt[k]) for k in (af.AF_CNT_EG1, af.AF_CNT_LF, af.AF_CNT_FLUX)] == \
                [int(cnt_or[k]) for k in (af.AF_CNT_EG1, af.AF_CNT_LF, af.AF_CNT_FLUX)]
            _close(out, ref, 1e-12)
    _flush(f"    L1(rho) vs exact: 128 cells {errs[128]:.3e}, 256 cells {errs[256]:.3e}")
    assert errs[256] < 2.5e-2 and errs[128] / errs[256] > 1.8
