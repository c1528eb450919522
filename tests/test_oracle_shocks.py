"""Pins of the oracle's transonic-shock linearisation (Algorithm 2) and shock-indicator blend
(Sec. 3.4).

Algorithm 2:
* data without a transonic sign change leave the method unchanged bit for bit;
* a transonic rarefaction (characteristic speeds diverging) is not flagged, a transonic shock
  (converging) is;
* a transonic shock moving to the left through a right-moving flow stalls when the full step is
  linearised at point values (the failure the paper illustrates), and moves at its
  Rankine-Hugoniot speed with Algorithm 2; in its monotone profile exactly one line of
  corners is flagged each step: ny corners, ny x-edges and 2 ny y-edges;
* the y direction is the transpose of the x direction.

Sec. 3.4:
* constant velocity and pressure (a contact) give theta = 1: no change at all;
* theta of a pressure bump in one cell, worked out by hand from the sensor's definition;
* where theta underflows to 0 the blended values are EG1 on piecewise constant data;
* the blend damps the oscillations behind a shock (smaller total variation).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I

G = I.GAMMA


def _shock_pair(M, s):
    """Left (upstream) and right states of a shock moving at speed s into the left state with
    upstream Mach number M relative to the shock (normal-shock relations)."""
    rL, pL = 1.0, 1.0
    cL = math.sqrt(G * pL / rL)
    wL = M * cL
    r = (G + 1) * M * M / ((G - 1) * M * M + 2)
    L = np.array([rL, wL + s, 0.0, pL])
    R = np.array([rL * r, wL / r + s, 0.0, pL * (1 + 2 * G / (G + 1) * (M * M - 1))])
    return L, R


def _jump_state(L, R, nx=100, ny=4, axis=0):
    """Piecewise constant data with the jump on the grid line through the domain centre
    (x = 0, or y = 0 for axis 1), outflow across the jump direction, periodic along it.  Point
    values on the jump take the mean state; averages are exact."""
    L, R = np.asarray(L, float), np.asarray(R, float)
    if axis == 0:
        grid = I.Grid(nx, ny, -1.0, 1.0, 0.0, 0.02 * ny, I.BC_OUTFLOW, I.BC_PERIODIC)
    else:
        grid = I.Grid(ny, nx, 0.0, 0.02 * ny, -1.0, 1.0, I.BC_PERIODIC, I.BC_OUTFLOW)
    M = 0.5 * (L + R)

    def prim(x, y, sites):
        c = x if axis == 0 else y
        W = np.where(c[None] < 0, L[:, None, None], R[:, None, None])
        if sites:
            W = np.where(np.isclose(c, 0.0)[None], M[:, None, None], W)
        return W

    sh = grid.shapes()
    K = prim(*grid.k_sites(), True)
    X = prim(*grid.x_sites(), True)
    Y = prim(*grid.y_sites(), True)
    avg = I.prim_to_cons(prim(*grid.cell_centres(), False), G)
    st = I.State(grid, G, np.ascontiguousarray(avg), np.ascontiguousarray(K),
                 np.ascontiguousarray(X), np.ascontiguousarray(Y))
    assert st.K.shape == sh["K"]
    return st


def _position(st, L, R, axis=0):
    """Where the density profile (mean over the periodic direction) crosses the mean of the
    two densities, by linear interpolation between cell centres."""
    g = st.grid
    rho = st.avg[0].mean(axis=0) if axis == 0 else st.avg[0].mean(axis=1)
    n, c0, h = (g.nx, g.x0, g.dx) if axis == 0 else (g.ny, g.y0, g.dy)
    xc = c0 + (np.arange(n) + 0.5) * h
    mid = 0.5 * (L[0] + R[0])
    k = np.where((rho[:-1] - mid) * (rho[1:] - mid) <= 0)[0][0]
    return xc[k] + (mid - rho[k]) / (rho[k + 1] - rho[k]) * h, rho


def test_transonic_pair_is_a_transonic_shock():
    L, R = _shock_pair(1.3, -0.2)
    cL, cR = math.sqrt(G * L[3] / L[0]), math.sqrt(G * R[3] / R[0])
    assert L[1] - cL > 0 > R[1] - cR  # u - c changes sign across the shock
    assert L[1] + cL > 0 and R[1] + cR > 0


def test_transonic_shock_moves_only_with_algorithm_2():
    L, R = _shock_pair(1.3, -0.2)
    t_end = 0.6
    res = {}
    for tsw in (False, True):
        st = _jump_state(L, R)
        e, n, cnt = oracle.run(st, t_end, 0.3, mode=oracle.MODE_AVG, limiter=True, tsw=tsw)
        assert e == oracle.OK and st.t == t_end
        x, rho = _position(st, L, R)
        res[tsw] = (x, n, cnt)
    exact = -0.2 * t_end
    dx = 2.0 / 100
    x_on, n_on, c_on = res[True]
    x_off, _, c_off = res[False]
    assert abs(x_on - exact) < 0.5 * dx, (x_on, exact)
    assert abs(x_off - exact) > 2 * dx, (x_off, exact)  # stalls behind the exact position
    assert c_off[5] == 0
    # one flagged corner line per step: ny corners + ny x-edges + 2 ny y-edges
    assert c_on[5] == 4 * 4 * n_on


def test_transonic_rarefaction_is_not_flagged():
    """Left state subsonic in u - c, right state supersonic (diverging characteristics)."""
    L = np.array([1.0, 0.5, 0.0, 1.0])
    R = np.array([0.6, 1.6, 0.0, 0.5])
    assert L[1] - math.sqrt(G * L[3] / L[0]) < 0 < R[1] - math.sqrt(G * R[3] / R[0])
    out = {}
    for tsw in (False, True):
        st = _jump_state(L, R, nx=40)
        e, n, cnt = oracle.run(st, 1e9, 0.3, max_steps=6, mode=oracle.MODE_AVG, limiter=True,
                               tsw=tsw)
        assert e == oracle.OK
        out[tsw] = (st, cnt)
    assert out[True][1][5] == 0
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(getattr(out[True][0], k), getattr(out[False][0], k))


def test_algorithm_2_changes_nothing_without_transonic_shocks():
    st = I.fourier_state(I.SEED_BASE + 7000, I.Grid(12, 10, 0.0, 1.0, 0.0, 1.0), G, 3)
    a, b = st.copy(), st.copy()
    e1, _, c1 = oracle.run(a, 1e9, 0.3, max_steps=3, mode=oracle.MODE_AVG)
    e2, _, c2 = oracle.run(b, 1e9, 0.3, max_steps=3, mode=oracle.MODE_AVG, tsw=True)
    assert e1 == e2 == oracle.OK and c2[5] == 0
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(getattr(a, k), getattr(b, k))


def test_transonic_shock_in_y_is_the_transpose():
    L, R = _shock_pair(1.3, -0.2)
    Ly = np.array([L[0], L[2], L[1], L[3]])
    Ry = np.array([R[0], R[2], R[1], R[3]])
    sx = _jump_state(L, R, nx=40)
    sy = _jump_state(Ly, Ry, nx=40, axis=1)
    ex, nx_, cx = oracle.run(sx, 1e9, 0.3, max_steps=8, mode=oracle.MODE_AVG, limiter=True,
                             tsw=True)
    ey, ny_, cy = oracle.run(sy, 1e9, 0.3, max_steps=8, mode=oracle.MODE_AVG, limiter=True,
                             tsw=True)
    assert ex == ey == oracle.OK and cx[5] == cy[5] > 0
    perm = [0, 2, 1, 3]
    scale = np.abs(sx.avg).max()
    assert np.abs(sy.avg[perm].transpose(0, 2, 1) - sx.avg).max() < 1e-12 * scale
    assert np.abs(sy.K[perm].transpose(0, 2, 1) - sx.K).max() < 1e-12 * scale
    assert np.abs(sy.Y[perm].transpose(0, 2, 1) - sx.X).max() < 1e-12 * scale


# ------------------------------------------------------------------------------------------
# Sec. 3.4
# ------------------------------------------------------------------------------------------
def test_shock_blend_leaves_contacts_alone():
    """Density variations in gas at rest under constant pressure (a steady contact): the
    energy and hence every primitive average's pressure is exactly 1, every pressure sensor
    is 0, theta = 1, and the blend changes nothing."""
    def fn(x, y):
        return np.stack([1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y),
                         0 * x, 0 * x, 1.0 + 0 * x])
    st = I.state_from_field(fn, I.Grid(12, 10, 0.0, 1.0, 0.0, 1.0), G, 3)
    for kind, i, j in ((oracle.KIND_K, 3, 4), (oracle.KIND_X, 0, 9), (oracle.KIND_Y, 11, 0)):
        e, th, f = oracle.indicators(st, kind, i, j)
        assert th == 1.0
    a, b = st.copy(), st.copy()
    oracle.run(a, 1e9, 0.3, max_steps=1, mode=oracle.MODE_AVG)
    oracle.run(b, 1e9, 0.3, max_steps=1, mode=oracle.MODE_AVG, shock=True)
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(getattr(a, k), getattr(b, k))


def _bump_state():
    """Gas at rest, rho = p = 1 at every point value, and one cell (5, 2) whose average holds
    p = 2: its primitive Simpson average is (1, 0, 0, 2), every other one (1, 0, 0, 1)."""
    grid = I.Grid(12, 6, 0.0, 1.0, 0.0, 1.0)
    st = I.uniform_state(grid, (1.0, 0.0, 0.0, 1.0))
    st.avg[3, 2, 5] = 2.0 / (G - 1)
    return st


def test_theta_worked_example():
    st = _bump_state()
    e, Uc, Ub = oracle.prep_cell(st, 5, 2)
    assert np.allclose(Ub, [1, 0, 0, 2], rtol=0, atol=1e-14)
    c1, c2 = math.sqrt(G * 1.0), math.sqrt(G * 2.0)
    # x-edges of row 2.  Line 6 (right face of the bump): sensors over cells (5,6,7) and
    # (4,5,6): |1-2+2|/5 = 1/5 and |1-4+1|/6 = 1/3; phi2 = 2^max(c(2), c(1)).
    th_a = math.exp(-(1 / 3) * 2 ** c2)
    # line 7: sensors over (6,7,8) = 0 and (5,6,7) = 1/5; phi2 over cells 6, 7 = 2^c(1).
    th_b = math.exp(-(1 / 5) * 2 ** c1)
    expect = {(oracle.KIND_X, 6, 2): th_a, (oracle.KIND_X, 5, 2): th_a,
              (oracle.KIND_X, 7, 2): th_b, (oracle.KIND_X, 4, 2): th_b,
              (oracle.KIND_X, 8, 2): 1.0, (oracle.KIND_X, 6, 3): 1.0,
              # y-edges of column 5: the same pattern along y
              (oracle.KIND_Y, 5, 2): th_a, (oracle.KIND_Y, 5, 3): th_a,
              (oracle.KIND_Y, 5, 4): th_b, (oracle.KIND_Y, 5, 1): th_b,
              (oracle.KIND_Y, 6, 2): 1.0,
              # corners: the smallest theta of the four edges next to them
              (oracle.KIND_K, 6, 2): th_a, (oracle.KIND_K, 7, 3): th_b,
              (oracle.KIND_K, 8, 3): 1.0, (oracle.KIND_K, 5, 4): th_b,
              (oracle.KIND_K, 5, 5): 1.0}
    for (kind, i, j), th in expect.items():
        e, got, f = oracle.indicators(st, kind, i, j)
        assert abs(got - th) < 1e-13, (kind, i, j, got, th)


def test_blend_is_eg1_where_theta_underflows():
    """Next to a strong, fast shock phi1 phi2 is large and theta < 1e-30, so 1 - theta = 1 and
    theta U_ho lies below rounding: the intermediate value is EG1 on piecewise constant data,
    linearised at the mean of the adjacent primitive averages, over dt/2."""
    L = np.array([1.0, 6.0, 0.0, 1.0])
    R = np.array([4.0, 1.5, 0.0, 60.0])
    st = _jump_state(L, R, nx=20)
    dt = 0.05 * st.grid.dx / oracle.max_speed(st)
    # the x-edges and corners on the lines next to the jump (y-edges sense pressure along y
    # only, which is constant here)
    for kind, i, j in ((oracle.KIND_X, 10, 1), (oracle.KIND_K, 10, 2), (oracle.KIND_K, 9, 0),
                       (oracle.KIND_X, 9, 3)):
        e, th, _ = oracle.indicators(st, kind, i, j)
        assert th < 1e-30
        e, h, f, _ = oracle.dof_update(st, kind, i, j, dt, mode=oracle.MODE_AVG, shock=True)
        assert e == oracle.OK
        if kind == oracle.KIND_K:
            cells = [(i - 1, j - 1), (i, j - 1), (i - 1, j), (i, j)]
        elif kind == oracle.KIND_X:
            cells = [(i - 1, j), (i, j)]
        else:
            cells = [(i, j - 1), (i, j)]
        Ut = np.mean([oracle.prep_cell(st, a, b)[2] for a, b in cells], axis=0)
        e, lo = oracle.dof_eg(st, 1, 1, kind, i, j, Ut, 0.5 * dt)
        assert e == oracle.OK
        assert np.allclose(h, lo, rtol=1e-14, atol=1e-14), (kind, h, lo)


def test_blend_damps_oscillations_behind_a_shock():
    L, R = _shock_pair(1.3, -0.2)
    tv = {}
    for shock in (False, True):
        st = _jump_state(L, R)
        e, n, _ = oracle.run(st, 0.6, 0.3, mode=oracle.MODE_AF3, limiter=True, shock=shock)
        assert e == oracle.OK
        _, rho = _position(st, L, R)
        tv[shock] = np.abs(np.diff(rho)).sum()
    exact = R[0] - L[0]
    assert tv[True] < 2.0 * exact < tv[False], tv
