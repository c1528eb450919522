"""Seeded synthetic inputs for the Active Flux step (shared by the oracle side and the HIP side).

This module holds *no* arithmetic of the method itself: only the initial data of the
workloads (closed-form fields, seeded noise and Fourier modes), their exact cell averages
by Gauss-Legendre quadrature, and the site geometry of the degrees of freedom.

Degrees of freedom (paper, Sec. 2, the paragraph introducing averages and point values):
  * cell averages of the conserved variables q = (rho, rho u, rho v, E), one per cell;
  * point values of the primitive variables U = (rho, u, v, p) at cell corners (kind K),
    vertical-edge midpoints (kind X) and horizontal-edge midpoints (kind Y).
Index conventions (0-based), with dx = (x1-x0)/nx:
  cell (i, j)  centre   (x0+(i+1/2)dx, y0+(j+1/2)dy)
  K (i, j)     corner   (x0+i dx,       y0+j dy)        lower-left corner of cell (i, j)
  X (i, j)     midpoint (x0+i dx,       y0+(j+1/2)dy)   left edge of cell (i, j)
  Y (i, j)     midpoint (x0+(i+1/2)dx,  y0+j dy)        bottom edge of cell (i, j)
Arrays are variable-major: avg (4, ny, nx); K (4, nky, nkx); X (4, ny, nkx); Y (4, nky, nx)
with nkx = nx + (0 if x is periodic else 1), nky likewise.

Seeds follow SplitMix64 (Steele, Lea, Flood 2014); uniform doubles are (z >> 11) * 2**-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4
BC_PERIODIC = 0
BC_OUTFLOW = 1
BC_WALL = 2
BC_INFLOW = 3
SEED_BASE = 250806273

# --------------------------------------------------------------------------------------
# SplitMix64
# --------------------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset..offset+n-1 of the SplitMix64 stream started at `seed` (uint64 array)."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n uniform doubles in [0, 1) from SplitMix64."""
    z = splitmix64(seed, n, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------------------
# Grid geometry
# --------------------------------------------------------------------------------------
@dataclass
class Grid:
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    # optional kind per side (left, right, bottom, top); None: bc_x on both x sides, bc_y on
    # both y sides.  A non-periodic axis needs bc_x / bc_y != BC_PERIODIC.
    sides: tuple | None = None
    # optional primitive inflow state per side (None where the side is not inflow)
    inflow: tuple | None = None

    def __post_init__(self):
        if self.sides is not None:
            s = tuple(int(k) for k in self.sides)
            assert len(s) == 4
            for ax, (lo, hi) in enumerate(((s[0], s[1]), (s[2], s[3]))):
                assert (lo == BC_PERIODIC) == (hi == BC_PERIODIC), "periodic must pair"
                kind = BC_PERIODIC if lo == BC_PERIODIC else BC_OUTFLOW
                if ax == 0:
                    self.bc_x = kind
                else:
                    self.bc_y = kind
            self.sides = s
            for k, kind in enumerate(s):
                if kind == BC_INFLOW:
                    assert self.inflow is not None and self.inflow[k] is not None

    def side_kinds(self) -> tuple:
        if self.sides is not None:
            return self.sides
        return (self.bc_x, self.bc_x, self.bc_y, self.bc_y)

    def inflow_state(self, side: int):
        if self.inflow is None:
            return None
        return self.inflow[side]

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny

    @property
    def nkx(self) -> int:
        return self.nx + (0 if self.bc_x == BC_PERIODIC else 1)

    @property
    def nky(self) -> int:
        return self.ny + (0 if self.bc_y == BC_PERIODIC else 1)

    def shapes(self):
        return dict(avg=(4, self.ny, self.nx), K=(4, self.nky, self.nkx),
                    X=(4, self.ny, self.nkx), Y=(4, self.nky, self.nx))

    def dof_count(self) -> int:
        """Number of DOF sites (each a 4-vector): averages + K + X + Y."""
        return (self.nx * self.ny + self.nkx * self.nky + self.nkx * self.ny
                + self.nx * self.nky)

    # site coordinates -----------------------------------------------------------------
    def cell_centres(self):
        xc = self.x0 + (np.arange(self.nx) + 0.5) * self.dx
        yc = self.y0 + (np.arange(self.ny) + 0.5) * self.dy
        return np.meshgrid(xc, yc)

    def k_sites(self):
        xs = self.x0 + np.arange(self.nkx) * self.dx
        ys = self.y0 + np.arange(self.nky) * self.dy
        return np.meshgrid(xs, ys)

    def x_sites(self):
        xs = self.x0 + np.arange(self.nkx) * self.dx
        ys = self.y0 + (np.arange(self.ny) + 0.5) * self.dy
        return np.meshgrid(xs, ys)

    def y_sites(self):
        xs = self.x0 + (np.arange(self.nx) + 0.5) * self.dx
        ys = self.y0 + np.arange(self.nky) * self.dy
        return np.meshgrid(xs, ys)


def prim_to_cons(W: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    """Conserved (rho, rho u, rho v, E) of primitive (rho, u, v, p), ideal gas (paper Sec. 2).

    Operation order is fixed (it is part of the input definition):
    E = p/(gamma-1) + 0.5*rho*(u*u + v*v).
    """
    rho, u, v, p = W[0], W[1], W[2], W[3]
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


@dataclass
class State:
    grid: Grid
    gamma: float
    avg: np.ndarray
    K: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    t: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    def copy(self) -> "State":
        return State(self.grid, self.gamma, self.avg.copy(), self.K.copy(), self.X.copy(),
                     self.Y.copy(), self.t, self.name, dict(self.meta))


def cell_average(fn, grid: Grid, gamma: float = GAMMA, n_gl: int = 6,
                 conserved: bool = True, rows_per_chunk: int = 256) -> np.ndarray:
    """n_gl x n_gl Gauss-Legendre cell averages of fn(x, y) -> (4, ...) primitive field.

    With conserved=True the average is taken of prim_to_cons(fn); else of fn itself.
    """
    g, w = np.polynomial.legendre.leggauss(n_gl)
    g = 0.5 * g
    w = 0.5 * w
    out = np.empty((4, grid.ny, grid.nx))
    xc = grid.x0 + (np.arange(grid.nx) + 0.5) * grid.dx
    for j0 in range(0, grid.ny, rows_per_chunk):
        j1 = min(grid.ny, j0 + rows_per_chunk)
        yc = grid.y0 + (np.arange(j0, j1) + 0.5) * grid.dy
        acc = np.zeros((4, j1 - j0, grid.nx))
        for a in range(n_gl):
            for b in range(n_gl):
                X, Yv = np.meshgrid(xc + g[a] * grid.dx, yc + g[b] * grid.dy)
                W = fn(X, Yv)
                acc += (w[a] * w[b]) * (prim_to_cons(W, gamma) if conserved else W)
        out[:, j0:j1, :] = acc
    return out


def state_from_field(fn, grid: Grid, gamma: float = GAMMA, n_gl: int = 6, name: str = "",
                     site_fn=None) -> State:
    """Averages by quadrature of fn, point values pointwise (site_fn defaults to fn)."""
    sf = site_fn or fn
    avg = cell_average(fn, grid, gamma, n_gl)
    K = np.asarray(sf(*grid.k_sites()), dtype=np.float64)
    X = np.asarray(sf(*grid.x_sites()), dtype=np.float64)
    Y = np.asarray(sf(*grid.y_sites()), dtype=np.float64)
    return State(grid, gamma, avg, K, X, Y, 0.0, name)


# --------------------------------------------------------------------------------------
# Workload fields
# --------------------------------------------------------------------------------------
def uniform_field(W0):
    W0 = np.asarray(W0, dtype=np.float64)

    def fn(x, y):
        return np.broadcast_to(W0[:, None, None] if np.ndim(x) == 2 else W0[:, None],
                               (4,) + np.shape(x)).copy()
    return fn


def uniform_state(grid: Grid, W0, gamma: float = GAMMA) -> State:
    """Constant admissible state: point values W0, averages prim_to_cons(W0) exactly."""
    W0 = np.asarray(W0, dtype=np.float64)
    Q0 = prim_to_cons(W0.reshape(4, 1), gamma).reshape(4)
    sh = grid.shapes()
    st = State(grid, gamma,
               np.broadcast_to(Q0[:, None, None], sh["avg"]).copy(),
               np.broadcast_to(W0[:, None, None], sh["K"]).copy(),
               np.broadcast_to(W0[:, None, None], sh["X"]).copy(),
               np.broadcast_to(W0[:, None, None], sh["Y"]).copy(), 0.0, "uniform")
    return st


# Shu-type isentropic vortex (the workload's vortex: strength eps at (xc, yc), background
# (1,1,1,1)).  Radial balance dp/dr = rho u_theta^2 / r with p = rho^gamma gives the
# temperature T = p/rho = 1 - (gamma-1) eps^2/(8 gamma pi^2) exp(1-r^2).
def shu_vortex_field(t: float = 0.0, eps: float = 5.0, centre=(5.0, 5.0), L: float = 10.0,
                     gamma: float = GAMMA, background=(1.0, 1.0, 1.0, 1.0)):
    rho0, u0, v0, p0 = background
    assert rho0 == 1.0 and p0 == 1.0, "closed form assumes rho0 = p0 = 1"

    def fn(x, y):
        # nearest periodic image of the vortex centre after translation by (u0 t, v0 t)
        dx = np.mod(x - centre[0] - u0 * t + 0.5 * L, L) - 0.5 * L
        dy = np.mod(y - centre[1] - v0 * t + 0.5 * L, L) - 0.5 * L
        r2 = dx * dx + dy * dy
        e = np.exp(0.5 * (1.0 - r2))
        du = -eps / (2.0 * math.pi) * e * dy
        dv = eps / (2.0 * math.pi) * e * dx
        T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * e * e
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return np.stack([rho, u0 + du, v0 + dv, p])
    return fn


def shu_vortex(n: int, t: float = 0.0, n_gl: int = 6, gamma: float = GAMMA) -> State:
    grid = Grid(n, n, 0.0, 10.0, 0.0, 10.0)
    return state_from_field(shu_vortex_field(t, gamma=gamma), grid, gamma, n_gl, f"shu{n}")


# Example 1 of the paper (Sec. 2): 1D density/pressure pulse, u = v = 0, on [0,1] in x with
# square cells in y (the solution is y-independent, so the y-extent is ny*dx).
def ex1_field():
    def fn(x, y):
        g = 1.0 + 0.5 * np.exp(-80.0 * (x - 0.5) ** 2)
        z = np.zeros_like(x)
        return np.stack([g, z, z, g.copy()])
    return fn


def ex1_state(nx: int, ny: int = 8, n_gl: int = 6) -> State:
    dx = 1.0 / nx
    grid = Grid(nx, ny, 0.0, 1.0, 0.0, ny * dx)
    return state_from_field(ex1_field(), grid, GAMMA, n_gl, f"ex1_{nx}")


# Example 2 of the paper (Sec. 2): compact travelling vortex on [0,1]^2, period 1.
# The printed swirl (1 - r^6) r^6 is read as (1 - r)^6 r^6: only that form balances the
# printed pressure polynomial (checked in the tests).
EX2_P_COEF = {36: 1 / 72, 35: -6 / 35, 34: 15 / 17, 33: -74 / 33, 32: 57 / 32, 31: 174 / 31,
              30: -269 / 15, 29: 450 / 29, 28: 153 / 8, 27: -1564 / 27, 26: 510 / 13,
              25: 204 / 5, 24: -1473 / 16, 23: 1014 / 23, 22: 1053 / 22, 21: -558 / 7,
              20: 783 / 20, 19: 54 / 19, 18: -38 / 9, 17: -222 / 17, 16: 609 / 32,
              15: -184 / 15, 14: 9 / 2, 13: -12 / 13, 12: 1 / 12}


def ex2_pressure_poly(r):
    r = np.asarray(r, dtype=np.float64)
    acc = sum(c * r ** k for k, c in EX2_P_COEF.items())
    return 1024.0 ** 2 * acc


def ex2_field(t: float = 0.0):
    rc, uc, vc, pc = 0.5, 1.0, 1.0, 0.1
    x0, y0, R = 0.5, 0.5, 0.4
    p1 = float(ex2_pressure_poly(np.array(1.0)))

    def fn(x, y):
        dx = np.mod(x - x0 - uc * t + 0.5, 1.0) - 0.5
        dy = np.mod(y - y0 - vc * t + 0.5, 1.0) - 0.5
        dist = np.sqrt(dx * dx + dy * dy)
        r = dist / R
        inside = r < 1.0
        rr = np.where(inside, r, 0.0)
        rho = rc + np.where(inside, 0.5 * (1.0 - rr * rr) ** 6, 0.0)
        sw = np.where(inside, 1024.0 * (1.0 - rr) ** 6 * rr ** 6, 0.0)
        safe = np.where(dist > 0, dist, 1.0)
        s = np.where(dist > 0, dy / safe, 0.0)
        c = np.where(dist > 0, dx / safe, 0.0)
        u = uc - sw * s
        v = vc + sw * c
        p = pc + np.where(inside, ex2_pressure_poly(rr) - p1, 0.0)
        return np.stack([rho, u, v, p])
    return fn


def ex2_state(n: int, n_gl: int = 6) -> State:
    grid = Grid(n, n, 0.0, 1.0, 0.0, 1.0)
    return state_from_field(ex2_field(0.0), grid, GAMMA, n_gl, f"ex2_{n}")


# Positivity stress (radial outflow towards near-vacuum at the centre) on [-1,1]^2, outflow.
def radial_field():
    def fn(x, y):
        r = np.sqrt(x * x + y * y)
        safe = np.where(r > 0, r, 1.0)
        u = np.where(r > 0, 2.0 * x / safe, 0.0)
        v = np.where(r > 0, 2.0 * y / safe, 0.0)
        return np.stack([np.ones_like(x), u, v, 0.4 * np.ones_like(x)])
    return fn


def radial_state(n: int = 2048, seed: int = SEED_BASE + 3000, n_gl: int = 4,
                 noise: float = 0.01) -> State:
    grid = Grid(n, n, -1.0, 1.0, -1.0, 1.0, BC_OUTFLOW, BC_OUTFLOW)
    st = state_from_field(radial_field(), grid, GAMMA, n_gl, f"radial{n}")
    off = 0
    for arr in (st.K, st.X, st.Y):
        m = arr[0].size
        xi_r = 2.0 * uniform01(seed, m, off) - 1.0
        xi_p = 2.0 * uniform01(seed, m, off + m) - 1.0
        off += 2 * m
        arr[0] *= (1.0 + noise * xi_r.reshape(arr[0].shape))
        arr[3] *= (1.0 + noise * xi_p.reshape(arr[3].shape))
    m = st.avg[0].size
    xi_r = (2.0 * uniform01(seed, m, off) - 1.0).reshape(st.avg[0].shape)
    xi_p = (2.0 * uniform01(seed, m, off + m) - 1.0).reshape(st.avg[0].shape)
    eint = cell_average(lambda x, y: radial_field()(x, y), grid, GAMMA, n_gl, conserved=False)[3] \
        / (GAMMA - 1.0)
    ekin = st.avg[3] - eint
    f = 1.0 + noise * xi_r
    st.avg[0] *= f
    st.avg[1] *= f
    st.avg[2] *= f
    st.avg[3] = ekin * f + eint * (1.0 + noise * xi_p)
    st.meta.update(seed=seed, noise=noise)
    return st


# Batched periodic grids with random Fourier-mode data on [0,1]^2.
def fourier_modes(seed: int, n_modes: int = 8):
    u = uniform01(seed, 4 * n_modes)
    m = np.floor(u[0:n_modes] * 9).astype(int) - 4
    n = np.floor(u[n_modes:2 * n_modes] * 9).astype(int) - 4
    # (0,0) is excluded: replace by (1,0)
    zero = (m == 0) & (n == 0)
    m[zero] = 1
    phi = 2.0 * math.pi * u[2 * n_modes:3 * n_modes]
    a = u[3 * n_modes:4 * n_modes] + 1e-12
    a = a / a.sum()
    return m, n, phi, a


def fourier_field(seed: int):
    modes = [fourier_modes(seed + 17 * k) for k in range(4)]
    amp = [0.2, 0.3, 0.3, 0.2]
    base = [1.0, 0.0, 0.0, 1.0]

    def fn(x, y):
        out = []
        for k in range(4):
            m, n, phi, a = modes[k]
            s = np.zeros_like(x)
            for q in range(len(a)):
                s = s + a[q] * np.cos(2.0 * math.pi * (m[q] * x + n[q] * y) + phi[q])
            out.append(base[k] + amp[k] * s)
        return np.stack(out)
    return fn


def fourier_tensor(seed: int, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """fourier_field(seed) on the tensor grid ys x xs, shape (4, len(ys), len(xs)).

    Each variable is base + amp * Re(sum_q a_q e^{i phi_q} e^{2 pi i m_q x} e^{2 pi i n_q y}),
    one (ny x 8) @ (8 x nx) complex product per variable."""
    amp = [0.2, 0.3, 0.3, 0.2]
    base = [1.0, 0.0, 0.0, 1.0]
    out = np.empty((4, len(ys), len(xs)))
    for k in range(4):
        m, n, phi, a = fourier_modes(seed + 17 * k)
        ex = np.exp(2j * math.pi * np.outer(xs, m))            # (nx, 8)
        ey = np.exp(2j * math.pi * np.outer(ys, n)) * (a * np.exp(1j * phi))  # (ny, 8)
        out[k] = base[k] + amp[k] * (ey @ ex.T).real
    return out


def fourier_state(seed: int, grid: Grid, gamma: float = GAMMA, n_gl: int = 4,
                  name: str = "") -> State:
    """state_from_field(fourier_field(seed), grid, gamma, n_gl) computed on tensor grids."""
    g, w = np.polynomial.legendre.leggauss(n_gl)
    g, w = 0.5 * g, 0.5 * w
    xc = grid.x0 + (np.arange(grid.nx) + 0.5) * grid.dx
    yc = grid.y0 + (np.arange(grid.ny) + 0.5) * grid.dy
    avg = np.zeros((4, grid.ny, grid.nx))
    for b in range(n_gl):
        for a in range(n_gl):
            W = fourier_tensor(seed, xc + g[a] * grid.dx, yc + g[b] * grid.dy)
            avg += (w[a] * w[b]) * prim_to_cons(W, gamma)
    xk = grid.x0 + np.arange(grid.nkx) * grid.dx
    yk = grid.y0 + np.arange(grid.nky) * grid.dy
    K = fourier_tensor(seed, xk, yk)
    X = fourier_tensor(seed, xk, yc)
    Y = fourier_tensor(seed, xc, yk)
    return State(grid, gamma, avg, K, X, Y, 0.0, name)


def batched_sizes(n_grids: int = 256, seed: int = SEED_BASE + 4000, lo: int = 64,
                  hi: int = 512):
    u = uniform01(seed, n_grids)
    return (lo + np.floor(u * (hi - lo + 1))).astype(int)


def batched_states(n_grids: int = 256, seed: int = SEED_BASE + 4000, lo: int = 64,
                   hi: int = 512, n_gl: int = 4, sizes=None):
    """The batched workload: periodic N x N grids on [0,1]^2, N ~ U{lo..hi}, grid g with the
    Fourier data of seed + 100 (g + 1)."""
    sizes = batched_sizes(n_grids, seed, lo, hi) if sizes is None else sizes
    out = []
    for g, N in enumerate(sizes):
        grid = Grid(int(N), int(N), 0.0, 1.0, 0.0, 1.0)
        out.append(fourier_state(seed + 100 * (g + 1), grid, GAMMA, n_gl, f"batch{g}_{N}"))
    return out


# Closed box [0,1]^2: a smooth field that is even about x = 0, 1 (rho, v, p) or odd (u), and
# likewise in y with v odd, so that it is the restriction of a mirror-symmetric field of
# period 2; random amplitudes of the modes cos / sin (k pi x) cos / sin (l pi y), k, l <= 2.
def mirror_field(seed: int):
    u = uniform01(seed, 36) - 0.5

    def fn(x, y):
        cx = [np.cos(k * math.pi * x) for k in range(3)]
        sx = [np.sin(k * math.pi * x) for k in range(3)]
        cy = [np.cos(l * math.pi * y) for l in range(3)]
        sy = [np.sin(l * math.pi * y) for l in range(3)]
        rho = 1.0 + 0.0 * x
        p = 1.0 + 0.0 * x
        uu = 0.0 * x
        vv = 0.0 * x
        q = 0
        for k in range(3):
            for l in range(3):
                if k + l > 0:
                    rho = rho + 0.15 * u[q] * cx[k] * cy[l]
                    p = p + 0.15 * u[q + 9] * cx[k] * cy[l]
                uu = uu + 0.3 * u[q + 18] * sx[k] * cy[l]
                vv = vv + 0.3 * u[q + 27] * cx[k] * sy[l]
                q += 1
        return np.stack([rho, uu, vv, p])
    return fn


def box_state(n: int, seed: int = SEED_BASE + 6000, sides=(2, 2, 2, 2), n_gl: int = 4,
              ny: int | None = None) -> State:
    """mirror_field(seed) on [0,1]^2 with the given side kinds (wall, or periodic pairs).  On a
    wall line the normal velocity of the point values is set to exactly 0."""
    ny = n if ny is None else ny
    grid = Grid(n, ny, 0.0, 1.0, 0.0, 1.0, sides=tuple(sides))
    st = state_from_field(mirror_field(seed), grid, GAMMA, n_gl, f"box{n}")
    if sides[0] == BC_WALL:
        st.K[1, :, 0] = 0.0
        st.X[1, :, 0] = 0.0
    if sides[1] == BC_WALL:
        st.K[1, :, -1] = 0.0
        st.X[1, :, -1] = 0.0
    if sides[2] == BC_WALL:
        st.K[2, 0, :] = 0.0
        st.Y[2, 0, :] = 0.0
    if sides[3] == BC_WALL:
        st.K[2, -1, :] = 0.0
        st.Y[2, -1, :] = 0.0
    st.meta.update(seed=seed)
    return st


# Shock reflection (Sec. 4.3): [0,4] x [0,1]; the state (1, 2.9, 0, 1/1.4) everywhere except
# on the top line y = 1, which holds the post-shock state; inflow at the left (the upstream
# state) and at the top (the post-shock state), a solid wall at the bottom, outflow at the
# right.  Point values on y = 1 and the top inflow take the post-shock state.
SRP_UP = (1.0, 2.9, 0.0, 1.0 / 1.4)
SRP_POST = (1.69997, 2.61934, -0.50632, 1.52819)


def shock_reflection_state(nx: int = 120, ny: int = 30) -> State:
    grid = Grid(nx, ny, 0.0, 4.0, 0.0, 1.0,
                sides=(BC_INFLOW, BC_OUTFLOW, BC_WALL, BC_INFLOW),
                inflow=(SRP_UP, None, None, SRP_POST))
    st = uniform_state(grid, SRP_UP)
    st.K[:, -1, :] = np.asarray(SRP_POST)[:, None]
    st.Y[:, -1, :] = np.asarray(SRP_POST)[:, None]
    st.name = f"shock_reflection_{nx}x{ny}"
    return st


# Shear layer on [0,1]^2: inner strip |y-1/2| < 1/4 has rho = 2, u = -0.5; outside rho = 1,
# u = +0.5; p = 2.5; v = 0.01 sin(4 pi x) + 1e-3 white noise per site.  The jumps lie on
# grid lines when ny is a multiple of 4; point values on a jump take the mean of the two
# one-sided primitive states.
def shear_state(n: int = 8192, seed: int = SEED_BASE + 5000) -> State:
    assert n % 4 == 0
    grid = Grid(n, n, 0.0, 1.0, 0.0, 1.0)

    def prim(x, y, on_jump=None):
        inner = np.abs(y - 0.5) < 0.25
        rho = np.where(inner, 2.0, 1.0)
        u = np.where(inner, -0.5, 0.5)
        if on_jump is not None:
            rho = np.where(on_jump, 1.5, rho)
            u = np.where(on_jump, 0.0, u)
        v = 0.01 * np.sin(4.0 * math.pi * x)
        return np.stack([rho, u, v, 2.5 * np.ones_like(x)])

    dy = grid.dy
    jline = lambda y: (np.abs(np.abs(y - 0.5) - 0.25) < 0.25 * dy)
    off = 0
    arrs = {}
    for name, (xs, ys) in (("K", grid.k_sites()), ("X", grid.x_sites()), ("Y", grid.y_sites())):
        W = prim(xs, ys, jline(ys))
        m = xs.size
        W[2] += 1e-3 * (2.0 * uniform01(seed, m, off) - 1.0).reshape(xs.shape)
        off += m
        arrs[name] = W
    # exact averages: jumps lie on cell faces, so each cell is one-sided; the average of
    # sin(4 pi x) over a cell is closed form.
    xc, yc = grid.cell_centres()
    W = prim(xc, yc)
    h = grid.dx
    W[2] = 0.01 * np.sin(4.0 * math.pi * xc) * np.sin(2.0 * math.pi * h) / (2.0 * math.pi * h)
    m = xc.size
    W[2] += 1e-3 * (2.0 * uniform01(seed, m, off) - 1.0).reshape(xc.shape)
    avg = prim_to_cons(W)
    return State(grid, GAMMA, avg, arrs["K"], arrs["X"], arrs["Y"], 0.0, f"shear{n}",
                 {"seed": seed})


# --------------------------------------------------------------------------------------
# Error norms (L1 = dx dy sum |q_h - q_ref| over cells, Linf = max)
# --------------------------------------------------------------------------------------
def norms(avg: np.ndarray, ref: np.ndarray, grid: Grid):
    d = np.abs(avg - ref)
    l1 = d.reshape(4, -1).sum(axis=1) * grid.dx * grid.dy
    linf = d.reshape(4, -1).max(axis=1)
    return l1, linf
