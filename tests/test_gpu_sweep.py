"""A seeded sweep over the combinations the other parity tests take one at a time: grid shapes
from 2 to 45 cells per side (one tile to six, ragged edges, cells from 3x as wide as high to 3x
as high as wide), every kind of side on each side (periodic pairs, outflow, solid wall, inflow),
the three linearisations, with and without the correction, with and without the positivity
limiter, in both precisions.  Each case runs three steps on the GPU and in the FP64 oracle;
tolerances as in the other parity tests (FP64 1e-12 * scale, FP32 bulk 1e-6 * scale)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I

pytestmark = pytest.mark.gpu

af = pytest.importorskip("paper_2508_06273_amd.af")

PER, OUT, WALL, INFLOW = I.BC_PERIODIC, I.BC_OUTFLOW, I.BC_WALL, I.BC_INFLOW


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases(n=24, seed=I.SEED_BASE + 9100):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx, ny = int(rng.integers(2, 46)), int(rng.integers(2, 46))
        aspect = float(np.exp(rng.uniform(np.log(1 / 3), np.log(3))))  # dy / dx
        dx = float(rng.uniform(0.02, 0.1))
        sides = []
        for axis in range(2):
            if rng.random() < 0.35:
                sides += [PER, PER]
            else:
                sides += [int(rng.choice([OUT, WALL, INFLOW])) for _ in range(2)]
        inflow = tuple((float(rng.uniform(0.8, 1.2)), float(rng.uniform(-0.3, 0.3)),
                        float(rng.uniform(-0.3, 0.3)), float(rng.uniform(0.8, 1.2)))
                       if s == INFLOW else None for s in sides)
        grid = I.Grid(nx, ny, 0.0, nx * dx, 0.0, ny * dx * aspect, sides=tuple(sides),
                      inflow=inflow if INFLOW in sides else None)
        out.append(dict(grid=grid, seed=seed + 1 + k, mode=int(rng.integers(0, 3)),
                        correction=bool(rng.random() < 0.7), limiter=bool(rng.random() < 0.5)))
    return out


CASES = _cases()


def _assert_close(out, ref, tol, label):
    scale = max(float(np.abs(ref.avg).max()), float(np.abs(ref.K).max()))
    d = {k: float(np.abs(out[k] - getattr(ref, k)).max()) for k in ("avg", "K", "X", "Y")}
    _flush(f"    {label}: achieved max|diff|/scale {max(d.values()) / scale:.3e} (gate {tol:g})")
    bad = {k: v for k, v in d.items() if v > tol * scale}
    assert not bad, f"{label}: {d} (tol {tol * scale:.3e})"


@pytest.mark.parametrize("k", range(len(CASES)))
def test_sweep_matches_oracle(k):
    c = CASES[k]
    g = c["grid"]
    label = (f"case {k}: {g.nx}x{g.ny} sides {g.side_kinds()} dy/dx {g.dy / g.dx:.2f} "
             f"mode {c['mode']} correction {c['correction']} limiter {c['limiter']}")
    _flush(f"[gpu] sweep {label}")
    st = I.fourier_state(c["seed"], g, I.GAMMA, 3)
    opts = dict(linearisation=c["mode"], correction=c["correction"], limiter=c["limiter"])
    outs = {}
    for prec in (0, 1):
        s = af.Solver.for_state(st, precision=prec, **opts)
        t, n = s.run(1e9, 0.3, 3)
        outs[prec] = (s.get_state(), t, n)
        s.close()
    e, n2, _ = oracle.run(st, 1e9, 0.3, max_steps=3, mode=c["mode"],
                          correction=c["correction"], limiter=c["limiter"])
    assert e == 0 and n2 == 3
    for prec, tol in ((0, 1e-12), (1, 1e-6)):
        # the time reached follows the dt of each step, taken from the wave speeds of the
        # path's own state: in FP32 bulk these differ from the oracle's at the FP32 rounding
        out, t, n = outs[prec]
        assert n == 3, (prec, n)
        assert abs(t - st.t) <= tol * abs(st.t), (prec, t, st.t)
        _assert_close(out, st, tol, f"prec {prec}")
