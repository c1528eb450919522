"""Pins of the oracle's flux limiting of the cell averages (paper Sec. 3.5).

The paper gives the form F_lim = gamma F_ho + (1 - gamma) F_lo per face with gamma in [0, 1] as
large as possible such that the cell averages stay admissible, and leaves the construction to
the literature.  The oracle follows the positivity-preserving flux limiting of Hu, Adams and
Shu (2013): Rusanov low-order fluxes of the t_n averages, and per face the smallest over its
two cells of the largest theta that keeps each cell's share Q_lo - 4 lambda s theta dF of the
update above the floors.  Pinned here: the theta solver against the closed-form roots, that
smooth runs are untouched bit for bit, conservation to rounding on a periodic grid with
limiting active, and positivity where the unlimited scheme fails.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I

G = 1.4


def _pressure(Q):
    return (G - 1.0) * (Q[3] - 0.5 * (Q[1] ** 2 + Q[2] ** 2) / Q[0])


def _closed_form_theta(Qlo, d):
    """Largest theta in [0,1] with rho >= er and p >= ep along Qlo + theta d: the density bound
    is linear; the pressure bound, multiplied by the (positive) density, is the quadratic
    (r + t dr)(E + t dE) - |m + t dm|^2 / 2 - ep/(g-1) (r + t dr) >= 0, whose first root in
    (0, 1] ends the admissible interval."""
    Qlo, d = np.asarray(Qlo, float), np.asarray(d, float)
    er = min(1e-13, Qlo[0])
    ep = min(1e-13, _pressure(Qlo))
    tmax = 1.0
    if d[0] < 0:
        tmax = min(tmax, (Qlo[0] - er) / -d[0])
    k = ep / (G - 1.0)
    c0 = Qlo[0] * Qlo[3] - 0.5 * (Qlo[1] ** 2 + Qlo[2] ** 2) - k * Qlo[0]
    c1 = Qlo[0] * d[3] + d[0] * Qlo[3] - (Qlo[1] * d[1] + Qlo[2] * d[2]) - k * d[0]
    c2 = d[0] * d[3] - 0.5 * (d[1] ** 2 + d[2] ** 2)
    roots = np.roots([c2, c1, c0]) if abs(c2) > 0 else np.array([-c0 / c1])
    roots = [r.real for r in roots if abs(r.imag) < 1e-12 and r.real > 0]
    if roots:
        tmax = min(tmax, min(roots))
    return tmax


@pytest.mark.parametrize("seed", range(8))
def test_theta_matches_closed_form(seed):
    rng = np.random.default_rng(seed)
    W = np.array([0.5 + rng.random(), rng.normal(), rng.normal(), 0.2 + rng.random()])
    Qlo = I.prim_to_cons(W.reshape(4, 1)).reshape(4)
    d = rng.normal(size=4) * np.array([1.0, 2.0, 2.0, 3.0])
    if seed % 2 == 0:
        d[0] = -abs(d[0]) * 2.0  # density-limited cases
    got = oracle.flux_theta(Qlo, d)
    ref = _closed_form_theta(Qlo, d)
    assert abs(got - ref) < 1e-13, (got, ref)
    Q = Qlo + got * d
    assert Q[0] >= min(1e-13, Qlo[0]) and _pressure(Q) >= min(1e-13, _pressure(Qlo))


def test_theta_is_one_when_admissible():
    Qlo = np.array([1.0, 0.2, -0.1, 2.5])
    assert oracle.flux_theta(Qlo, np.array([0.01, -0.02, 0.03, 0.05])) == 1.0
    assert oracle.flux_theta(Qlo, np.zeros(4)) == 1.0


@pytest.mark.parametrize("mode", [0, 1])
def test_smooth_runs_unchanged_bitwise(mode):
    """Where no limiting is needed every gamma is 1 and the step is the unlimited one, bit for
    bit (config 1's vortex, a Fourier state with outflow sides)."""
    for st in (I.shu_vortex(24),
               I.state_from_field(I.fourier_field(3), I.Grid(20, 14, 0.0, 1.0, 0.0, 0.7, 1, 1),
                                  I.GAMMA, 3)):
        a, b = st.copy(), st.copy()
        e1, n1, c1 = oracle.run(a, 1e9, 0.3, max_steps=6, mode=mode)
        e2, n2, c2 = oracle.run(b, 1e9, 0.3, max_steps=6, mode=mode, flux_limiter=True)
        assert e1 == e2 == 0 and n1 == n2 == 6 and c2[6] == 0
        for k in ("avg", "K", "X", "Y"):
            assert np.array_equal(getattr(a, k), getattr(b, k)), k


def _divergent_state(n):
    """Periodic 1D-like data flowing apart from x = 0 (u = 2 sin 2 pi x): the centre empties
    towards vacuum."""
    def fn(x, y):
        return np.stack([np.ones_like(x), 2.0 * np.sin(2 * math.pi * x), 0.1 * np.cos(2 * math.pi * y),
                         0.4 * np.ones_like(x)])
    return I.state_from_field(fn, I.Grid(n, n, 0.0, 1.0, 0.0, 1.0), I.GAMMA, 3)


def test_conservation_with_limiting_active():
    st = _divergent_state(24)
    m0 = st.avg.reshape(4, -1).sum(axis=1)
    e, n, cnt = oracle.run(st, 1e9, 0.3, max_steps=60, mode=1, limiter=True, flux_limiter=True)
    assert e == 0 and n == 60
    assert cnt[6] > 0  # some faces were limited
    m1 = st.avg.reshape(4, -1).sum(axis=1)
    assert np.abs(m1 - m0).max() <= 1e-13 * np.abs(m0).max() * 60
    rho = st.avg[0]
    assert (rho > 0).all() and (_pressure(st.avg) > 0).all()


def test_limiting_keeps_averages_admissible_where_unlimited_fails():
    """The radial outflow towards near-vacuum (config 3's data on 32^2): without flux limiting
    a cell average loses positivity at step 137; with it, 600 steps keep every average
    admissible."""
    st = I.radial_state(32, n_gl=3)
    a = st.copy()
    e, n, _ = oracle.run(a, 1e9, 0.3, max_steps=300, mode=1, limiter=True)
    assert e == oracle.ERR_NONPHYSICAL and n < 300
    b = st.copy()
    e, n, cnt = oracle.run(b, 1e9, 0.3, max_steps=300, mode=1, limiter=True, flux_limiter=True)
    assert e == 0 and n == 300 and cnt[6] > 0
    assert (b.avg[0] > 0).all() and (_pressure(b.avg) > 0).all()
