"""Pins of the oracle's solid-wall and inflow boundaries (paper Sec. 4.3).

* A closed box with solid walls is the restriction of a periodic domain of twice the size whose
  data are mirror images about the walls (normal velocity odd, everything else even): the wall
  ghost rule (ghost averages and point values are the mirror images of the interior ones, with
  the normal velocity negated) must reproduce that periodic run on the box, DOF by DOF, in the
  linearisations whose intermediate state is built from point values (Algorithm 1 and the
  simplified method).  The periodic run shares none of the boundary code.
* With the averaged linearisation, a DOF on a wall line is linearised at its own point value
  (the paper's remark on reflecting boundaries): there it must coincide with the simplified
  method, and only there.
* Inflow: a uniform state whose inflow sides carry the same state stays uniform; and one step
  with inflow ghost data equals one step on a domain extended upstream by a region that holds
  the inflow state (the ghost point values, the ghost cells' centre values and averages are
  then the same numbers).
"""
import numpy as np
import pytest

import oracle
from paper_2508_06273_amd import inputs as I

G = I.GAMMA
WALL, INFLOW, OUTFLOW, PER = I.BC_WALL, I.BC_INFLOW, I.BC_OUTFLOW, I.BC_PERIODIC


def _mirror(a, axis, n, line, var):
    """Extend array `a` (variable axis 0) across index n on `axis` by its mirror image with
    variable `var` negated; the result has period 2n."""
    a = np.moveaxis(a, axis, -1)
    if line:
        ext = a[..., n - 1:0:-1].copy()
        base = a[..., :n + 1]
    else:
        ext = a[..., ::-1].copy()
        base = a
    ext[var] = -ext[var]
    out = np.concatenate([base, ext], axis=-1)
    return np.ascontiguousarray(np.moveaxis(out, -1, axis))


def _doubled(st, mx, my):
    """The periodic mirror-symmetric state on [0, 2] in each mirrored axis."""
    g = st.grid
    avg, K, X, Y = st.avg, st.K, st.X, st.Y
    if mx:
        avg = _mirror(avg, 2, g.nx, False, 1)
        K = _mirror(K, 2, g.nx, True, 1)
        X = _mirror(X, 2, g.nx, True, 1)
        Y = _mirror(Y, 2, g.nx, False, 1)
    if my:
        avg = _mirror(avg, 1, g.ny, False, 2)
        K = _mirror(K, 1, g.ny, True, 2)
        X = _mirror(X, 1, g.ny, False, 2)
        Y = _mirror(Y, 1, g.ny, True, 2)
    grid = I.Grid(g.nx * (2 if mx else 1), g.ny * (2 if my else 1), g.x0,
                  g.x1 + (g.x1 - g.x0) * (1 if mx else 0), g.y0,
                  g.y1 + (g.y1 - g.y0) * (1 if my else 0))
    return I.State(grid, st.gamma, avg, K, X, Y)


def _quadrant(big, st):
    g = st.grid
    return dict(avg=big.avg[:, :g.ny, :g.nx], K=big.K[:, :g.nky, :g.nkx],
                X=big.X[:, :g.ny, :g.nkx], Y=big.Y[:, :g.nky, :g.nx])


def _advance(st, dt, steps, **kw):
    for _ in range(steps):
        e, _ = oracle.step(st, dt, **kw)
        assert e == oracle.OK
    return st


@pytest.mark.parametrize("sides,n,ny,mode", [
    ((WALL, WALL, WALL, WALL), 10, 10, oracle.MODE_AF3),
    ((WALL, WALL, WALL, WALL), 9, 7, oracle.MODE_SIMPLE),
    ((WALL, WALL, PER, PER), 8, 6, oracle.MODE_AF3),
    ((PER, PER, WALL, WALL), 6, 9, oracle.MODE_AF3),
])
def test_closed_box_equals_mirrored_periodic_domain(sides, n, ny, mode):
    st = I.box_state(n, sides=sides, ny=ny)
    mx, my = sides[0] == WALL, sides[2] == WALL
    big = _doubled(st, mx, my)
    # the doubled data really are mirror images (checked on the constructed arrays)
    q = _quadrant(big, st)
    for k in ("avg", "K", "X", "Y"):
        assert np.array_equal(q[k], getattr(st, k))
    dt = 0.3 * min(st.grid.dx, st.grid.dy) / oracle.max_speed(st)
    assert dt == 0.3 * min(big.grid.dx, big.grid.dy) / oracle.max_speed(big)
    _advance(st, dt, 4, mode=mode)
    _advance(big, dt, 4, mode=mode)
    q = _quadrant(big, st)
    scale = max(np.abs(st.avg).max(), np.abs(st.K).max())
    for k in ("avg", "K", "X", "Y"):
        err = np.abs(getattr(st, k) - q[k]).max()
        assert err < 1e-12 * scale, (k, err)
    # the evolved normal velocity on the walls stays zero up to rounding
    if mx:
        assert np.abs(st.K[1, :, 0]).max() < 1e-13 and np.abs(st.X[1, :, -1]).max() < 1e-13
    if my:
        assert np.abs(st.K[2, 0, :]).max() < 1e-13 and np.abs(st.Y[2, -1, :]).max() < 1e-13


def test_closed_box_conserves_mass_and_energy():
    """Walls let no mass or energy through: the face fluxes on a wall line carry only the
    pressure term, so the totals of rho and E stay constant to rounding."""
    st = I.box_state(12, seed=I.SEED_BASE + 6100)
    m0 = st.avg.sum(axis=(1, 2))
    e, n, _ = oracle.run(st, 1e9, 0.3, max_steps=12, mode=oracle.MODE_AVG)
    assert e == oracle.OK and n == 12
    m1 = st.avg.sum(axis=(1, 2))
    assert abs(m1[0] - m0[0]) < 1e-12 * abs(m0[0])
    assert abs(m1[3] - m0[3]) < 1e-12 * abs(m0[3])


@pytest.mark.parametrize("kind,i,j,on_wall", [
    (oracle.KIND_K, 0, 3, True), (oracle.KIND_K, 10, 0, True), (oracle.KIND_K, 0, 0, True),
    (oracle.KIND_X, 10, 4, True), (oracle.KIND_Y, 5, 0, True), (oracle.KIND_Y, 2, 10, True),
    (oracle.KIND_K, 4, 5, False), (oracle.KIND_X, 1, 4, False), (oracle.KIND_Y, 0, 1, False),
    (oracle.KIND_X, 5, 0, False), (oracle.KIND_Y, 0, 4, False),
])
def test_averaged_linearisation_on_wall_uses_point_value(kind, i, j, on_wall):
    """Mode AVG on a wall line is the simplified method (intermediate state linearised at
    U^n); everywhere else it is the mean of the adjacent averages, which differs.  X sites on
    the bottom wall row and Y sites on the left wall column are not on a wall line."""
    st = I.box_state(10, seed=I.SEED_BASE + 6200)
    dt = 0.2 * st.grid.dx / oracle.max_speed(st)
    e1, h1, f1, _ = oracle.dof_update(st, kind, i, j, dt, mode=oracle.MODE_AVG)
    e2, h2, f2, _ = oracle.dof_update(st, kind, i, j, dt, mode=oracle.MODE_SIMPLE)
    assert e1 == e2 == oracle.OK
    if on_wall:
        assert np.array_equal(h1, h2) and np.array_equal(f1, f2)
    else:
        assert np.abs(h1 - h2).max() > 1e-9


def test_inflow_preserves_matching_uniform_state():
    W0 = (1.0, 2.9, 0.0, 1.0 / 1.4)
    grid = I.Grid(12, 6, 0.0, 4.0, 0.0, 1.0, sides=(INFLOW, OUTFLOW, WALL, INFLOW),
                  inflow=(W0, None, None, W0))
    st = I.uniform_state(grid, W0)
    ref = st.copy()
    e, n, _ = oracle.run(st, 1e9, 0.4, max_steps=6)
    assert e == oracle.OK and n == 6
    for k in ("avg", "K", "X", "Y"):
        assert np.abs(getattr(st, k) - getattr(ref, k)).max() < 1e-13, k


def _ramp_field(W_in):
    W_in = np.asarray(W_in, dtype=np.float64)

    def fn(x, y):
        b = np.where(x > 0.4, ((x - 0.4) / 0.6) ** 4, 0.0)
        out = np.stack([np.full_like(x, W_in[k]) for k in range(4)])
        out[0] = out[0] + 0.3 * b * (1.0 + 0.5 * np.sin(2 * np.pi * y))
        out[1] = out[1] - 0.4 * b * np.cos(2 * np.pi * y)
        out[2] = out[2] + 0.2 * b * np.sin(2 * np.pi * y)
        out[3] = out[3] + 0.2 * b
        return out
    return fn


@pytest.mark.parametrize("mode", [oracle.MODE_AF3, oracle.MODE_AVG, oracle.MODE_SIMPLE])
def test_inflow_step_equals_upstream_extended_domain(mode):
    W_in = (1.0, 2.0, 0.1, 0.5)
    n, ext = 16, 4
    fn = _ramp_field(W_in)
    grid = I.Grid(n, 8, 0.0, 1.0, 0.0, 1.0, sides=(INFLOW, OUTFLOW, PER, PER),
                  inflow=(W_in, None, None, None))
    st = I.state_from_field(fn, grid, G, 4)
    gx = I.Grid(n + ext, 8, -ext / n, 1.0, 0.0, 1.0, sides=(OUTFLOW, OUTFLOW, PER, PER))
    big = I.state_from_field(fn, gx, G, 4)
    # the upstream region holds the inflow state (point values exactly, averages to rounding)
    assert np.array_equal(big.K[:, :, :ext + 2], np.broadcast_to(
        np.asarray(W_in)[:, None, None], big.K[:, :, :ext + 2].shape))
    dt = 0.3 * grid.dx / oracle.max_speed(big)
    _advance(st, dt, 1, mode=mode)
    _advance(big, dt, 1, mode=mode)
    scale = max(np.abs(st.avg).max(), np.abs(st.K).max())
    for k, sl in (("avg", np.s_[:, :, ext:]), ("K", np.s_[:, :, ext:]),
                  ("X", np.s_[:, :, ext:]), ("Y", np.s_[:, :, ext:])):
        err = np.abs(getattr(st, k) - getattr(big, k)[sl]).max()
        assert err < 1e-13 * scale, (k, err)
    # the step did change the interior
    assert np.abs(st.K - I.state_from_field(fn, grid, G, 4).K).max() > 1e-4


def test_inflow_ghost_cell_centre_is_inflow_state():
    """The centre value of a ghost cell beyond an inflow side is the inflow state itself, also
    where the boundary point values differ from it; the ghost's primitive average is the
    Simpson average of its nine nodes."""
    W_in = np.array([1.3, 0.7, -0.2, 0.9])
    grid = I.Grid(6, 5, 0.0, 1.0, 0.0, 1.0, sides=(INFLOW, OUTFLOW, WALL, OUTFLOW),
                  inflow=(tuple(W_in), None, None, None))
    st = I.fourier_state(I.SEED_BASE + 6300, grid, G, 3)
    e, Uc, Ub = oracle.prep_cell(st, -1, 2)
    assert np.array_equal(Uc, W_in)
    K, X, Y = st.K, st.X, st.Y
    corners = 2 * W_in + K[:, 2, 0] + K[:, 3, 0]
    edges = W_in + X[:, 2, 0] + 2 * W_in
    nodes = (corners + 4 * edges + 16 * W_in) / 36
    assert np.allclose(Ub, nodes, rtol=0, atol=1e-15)
    # a corner ghost beyond the inflow side and the bottom wall: inflow wins
    e, Uc, _ = oracle.prep_cell(st, -1, -1)
    assert np.array_equal(Uc, W_in)


def test_wall_ghost_cell_is_mirror_of_first_cell():
    """A ghost cell beyond a wall is the mirror image of the cell it faces: its centre value
    and primitive average are that cell's with the normal velocity negated, exactly, and its
    reconstruction at a point is the facing cell's at the reflected point (also with a
    non-zero normal velocity on the wall line, where the two differ from a reconstruction
    through the ghost's own nodes)."""
    st = I.fourier_state(I.SEED_BASE + 6400, I.Grid(8, 7, 0.0, 1.0, 0.0, 0.7,
                                                    sides=(WALL, WALL, WALL, WALL)), G, 3)
    g = st.grid
    for (gi, gj), (ii, jj), var in (((-1, 3), (0, 3), 1), ((8, 5), (7, 5), 1),
                                    ((2, -1), (2, 0), 2), ((4, 7), (4, 6), 2)):
        _, Ucg, Ubg = oracle.prep_cell(st, gi, gj)
        _, Uci, Ubi = oracle.prep_cell(st, ii, jj)
        f = np.ones(4)
        f[var] = -1
        assert np.array_equal(Ucg, f * Uci) and np.array_equal(Ubg, f * Ubi)
        # a point of the ghost cell and its reflection about the wall line
        xg = g.x0 + (gi + 0.3) * g.dx
        yg = g.y0 + (gj + 0.8) * g.dy
        if var == 1:
            xw = g.x0 if gi < 0 else g.x1
            xr, yr = 2 * xw - xg, yg
        else:
            yw = g.y0 if gj < 0 else g.y1
            xr, yr = xg, 2 * yw - yg
        _, vg = oracle.eval_recon(st, gi, gj, xg, yg)
        _, vi = oracle.eval_recon(st, ii, jj, xr, yr)
        assert np.array_equal(vg, f * vi)
    # corner ghost beyond two walls: both velocity components negated
    _, Ucg, _ = oracle.prep_cell(st, -1, -1)
    _, Uci, _ = oracle.prep_cell(st, 0, 0)
    assert np.array_equal(Ucg, Uci * np.array([1, -1, -1, 1]))


def test_shock_reflection_states_are_consistent():
    """The shock-reflection problem's two given states are linked by an oblique shock at
    29 degrees (the exact solution's incident shock); the reflected state behind the second
    shock, which turns the flow back parallel to the wall, is the standard one."""
    import math
    import exact_shock as ES
    up = np.array(I.SRP_UP)
    post = ES.turned_state(up, math.radians(29.0), -1)
    assert np.allclose(post, I.SRP_POST, rtol=2e-5, atol=2e-5), post
    theta = -math.atan2(I.SRP_POST[2], I.SRP_POST[1])
    beta = ES.weak_shock_angle(np.array(I.SRP_POST), theta)
    refl = ES.turned_state(np.array(I.SRP_POST), beta, +1)
    assert abs(refl[2]) < 1e-12
    # reflected shock at about 23.3 degrees to the wall; region 3 about (2.687, 2.401, 0, 2.934)
    assert abs(math.degrees(beta - theta) - 23.28) < 0.02
    assert np.allclose(refl, [2.687, 2.401, 0.0, 2.934], atol=2e-3), refl


# Four constant states (lower left, lower right, upper left, upper right) that collide, with
# velocities normal to the horizontal walls in the cells next to them.
_QUAD = (np.array([1.0, 1.3, 1.3, 0.7]), np.array([1.8, -0.1, 1.3, 2.0]),
         np.array([1.8, 1.3, -0.1, 2.0]), np.array([2.5, -0.2, -0.2, 3.0]))


def _quadrant_state(grid, xs, ys):
    """_QUAD meeting at (xs, ys); a point value on a dividing line takes the mean of the states
    on either side."""
    def prim(x, y, sites):
        W = np.zeros((4,) + np.shape(x))
        for q, (r, t) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
            wx = (x > xs) * 1.0 if r else (x < xs) * 1.0
            wy = (y > ys) * 1.0 if t else (y < ys) * 1.0
            if sites:
                wx = wx + 0.5 * (x == xs)
                wy = wy + 0.5 * (y == ys)
            W += _QUAD[q].reshape((4,) + (1,) * np.ndim(x)) * (wx * wy)[None]
        return W

    avg = I.cell_average(lambda x, y: prim(x, y, False), grid, G, 4)
    return I.State(grid, G, avg, prim(*grid.k_sites(), True), prim(*grid.x_sites(), True),
                   prim(*grid.y_sites(), True))


def _flip_y(st):
    """The problem mirrored about the horizontal mid-line: rows reversed, v negated, bottom and
    top sides exchanged."""
    g = st.grid
    sides = (g.sides[0], g.sides[1], g.sides[3], g.sides[2])
    inflow = None
    if g.inflow is not None:
        def neg(w):
            return None if w is None else (w[0], w[1], -w[2], w[3])
        inflow = (neg(g.inflow[0]), neg(g.inflow[1]), neg(g.inflow[3]), neg(g.inflow[2]))
    grid = I.Grid(g.nx, g.ny, g.x0, g.x1, g.y0, g.y1, sides=sides, inflow=inflow)
    out = []
    for a in (st.avg, st.K, st.X, st.Y):
        b = a[:, ::-1, :].copy()
        b[2] = -b[2]
        out.append(np.ascontiguousarray(b))
    return I.State(grid, st.gamma, *out)


@pytest.mark.parametrize("mode", [oracle.MODE_AF3, oracle.MODE_AVG, oracle.MODE_SIMPLE])
def test_wall_problem_is_mirror_equivariant(mode):
    """A problem and its mirror image about the horizontal mid-line (walls below and above,
    inflow on the left, a wall on the right) evolve into mirror images, with the positivity
    limiter (Algorithm 3) and the Sec. 3.4 blend on.  The Sec. 3.4 low-order value is EG1 on
    piecewise constant data, which jumps where its foot point crosses a grid line: on a wall
    the mean of the adjacent averages has zero normal velocity, so the foot point lies on the
    wall line and the value is the mean over both sides.  A mean that kept a rounding residue
    in v would put the foot point on one side or the other depending on the wall's
    orientation, and the two runs would differ at O(1) there."""
    grid = I.Grid(29, 18, 0.0, 1.0, 0.0, 0.9, sides=(INFLOW, WALL, WALL, WALL),
                  inflow=((1.5, 0.1, -0.05, 1.8), None, None, None))
    st = _quadrant_state(grid, 0.55, 0.4)
    fl = _flip_y(st)
    kw = dict(mode=mode, limiter=True, shock=True)
    dt = 0.3 * min(grid.dx, grid.dy) / oracle.max_speed(st, **kw)
    assert abs(dt - 0.3 * min(grid.dx, grid.dy) / oracle.max_speed(fl, **kw)) <= 1e-15 * dt
    _advance(st, dt, 3, **kw)
    _advance(fl, dt, 3, **kw)
    back = _flip_y(fl)
    scale = max(np.abs(st.avg).max(), np.abs(st.K).max())
    for k in ("avg", "K", "X", "Y"):
        err = np.abs(getattr(st, k) - getattr(back, k)).max()
        assert err < 1e-12 * scale, (k, err)
