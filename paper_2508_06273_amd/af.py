"""Thin ctypes binding of libaf.so (C ABI in include/af.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy arrays to
pointers and error codes to exceptions.  It raises if the library has not been built
(see paper_2508_06273_amd/build.py) -- there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaf.so")

AF_OK, AF_ERR_INVALID_ARG, AF_ERR_NONPHYSICAL, AF_ERR_CFL, AF_ERR_DEVICE, AF_ERR_OOM = \
    0, -1, -2, -3, -4, -5
AF_BC_PERIODIC, AF_BC_OUTFLOW, AF_BC_WALL, AF_BC_INFLOW = 0, 1, 2, 3
AF_SIDE_LEFT, AF_SIDE_RIGHT, AF_SIDE_BOTTOM, AF_SIDE_TOP = 0, 1, 2, 3
AF_OPT_PRECISION, AF_OPT_LINEARISATION, AF_OPT_CORRECTION, AF_OPT_LIMITER, \
    AF_OPT_GRAPH_STEPS, AF_OPT_TIMING, AF_OPT_AUTOTUNE, AF_OPT_TILE_ORDER, \
    AF_OPT_UPDATE_THREADS, AF_OPT_TRANSONIC, AF_OPT_SHOCK_LIMITER, AF_OPT_FLUX_LIMITER, \
    AF_OPT_STEP_KERNEL, AF_OPT_SYNC_TIMEOUT_US = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14
AF_ORDER_XCD, AF_ORDER_LINEAR, AF_ORDER_GRIDS = 0, 1, 2
AF_STEP_SPLIT, AF_STEP_PERSISTENT = 0, 1
AF_PREC_FP64, AF_PREC_FP32 = 0, 1
AF_LIN_AF3, AF_LIN_AVG, AF_LIN_SIMPLE = 0, 1, 2
AF_CNT_EG1, AF_CNT_LF, AF_CNT_CENTRE, AF_CNT_INNER, AF_CNT_STEPS, AF_CNT_TSW, AF_CNT_FLUX = \
    0, 1, 2, 3, 4, 5, 6
AF_NCOUNTERS = 8

# every symbol include/af.h declares
EXPORTS = ["af_create", "af_set_option", "af_set_stream", "af_set_state", "af_get_state",
           "af_step", "af_run", "af_get_counters", "af_destroy", "af_last_error",
           "af_dof_count", "af_get_timing", "af_create_batch", "af_batch_size",
           "af_set_state_grid", "af_get_state_grid", "af_get_grid_info", "af_get_option",
           "af_set_inflow", "af_set_state_device", "af_get_state_device",
           "af_step_noalloc", "af_get_totals"]


class AfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"af error {code}: {msg}")
        self.code = code


class Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("x0", ct.c_double),
                ("x1", ct.c_double), ("y0", ct.c_double), ("y1", ct.c_double)]


class Bc(ct.Structure):
    _fields_ = [("left", ct.c_int32), ("right", ct.c_int32), ("bottom", ct.c_int32),
                ("top", ct.c_int32)]


_lib = None
_D = ct.POINTER(ct.c_double)
_H = ct.c_void_p


def load(path: str = LIB_PATH):
    """Load libaf.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run paper_2508_06273_amd/build.py")
    L = ct.CDLL(path)
    L.af_create.argtypes = [ct.POINTER(Grid), ct.c_double, ct.POINTER(Bc), ct.POINTER(_H)]
    L.af_set_option.argtypes = [_H, ct.c_int, ct.c_int64]
    L.af_set_stream.argtypes = [_H, ct.c_void_p]
    L.af_set_state.argtypes = [_H, _D, _D, _D, _D, ct.c_double]
    L.af_get_state.argtypes = [_H, _D, _D, _D, _D, _D]
    L.af_step.argtypes = [_H, ct.c_double]
    L.af_run.argtypes = [_H, ct.c_double, ct.c_double, ct.c_int64, _D,
                         ct.POINTER(ct.c_int64)]
    L.af_get_counters.argtypes = [_H, ct.POINTER(ct.c_int64)]
    L.af_get_totals.argtypes = [_H, ct.c_int32, _D]
    L.af_destroy.argtypes = [_H]
    L.af_destroy.restype = None
    L.af_last_error.argtypes = [_H]
    L.af_last_error.restype = ct.c_char_p
    L.af_dof_count.argtypes = [_H]
    L.af_dof_count.restype = ct.c_int64
    L.af_get_timing.argtypes = [_H, ct.POINTER(ct.c_double)]
    L.af_get_timing.restype = ct.c_int
    L.af_create_batch.argtypes = [ct.c_int32, ct.POINTER(Grid), ct.c_double, ct.POINTER(Bc),
                                  ct.POINTER(_H)]
    L.af_batch_size.argtypes = [_H]
    L.af_batch_size.restype = ct.c_int32
    L.af_set_state_grid.argtypes = [_H, ct.c_int32, _D, _D, _D, _D, ct.c_double]
    L.af_get_state_grid.argtypes = [_H, ct.c_int32, _D, _D, _D, _D, _D]
    L.af_get_grid_info.argtypes = [_H, ct.c_int32, _D, ct.POINTER(ct.c_int64)]
    L.af_get_option.argtypes = [_H, ct.c_int, ct.POINTER(ct.c_int64)]
    L.af_set_inflow.argtypes = [_H, ct.c_int32, ct.c_int32, _D]
    L.af_set_state_device.argtypes = [_H, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, ct.c_double]
    L.af_get_state_device.argtypes = [_H, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, _D]
    L.af_step_noalloc.argtypes = [ct.POINTER(Grid), ct.c_double, ct.POINTER(Bc), _D, ct.c_int32,
                                  ct.c_int32, ct.c_int32, ct.c_int32] + [ct.c_void_p] * 8 + \
        [ct.c_int64, ct.c_int64, ct.c_double, ct.c_void_p, ct.POINTER(ct.c_int64)]
    for name in ("af_create", "af_set_option", "af_set_stream", "af_set_state",
                 "af_get_state", "af_step", "af_run", "af_get_counters", "af_create_batch",
                 "af_set_state_grid", "af_get_state_grid", "af_get_grid_info",
                 "af_get_option", "af_set_inflow", "af_set_state_device",
                 "af_get_state_device", "af_step_noalloc"):
        getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _shapes(nx, ny, nkx, nky):
    return dict(avg=(4, ny, nx), K=(4, nky, nkx), X=(4, ny, nkx), Y=(4, nky, nx))


def _sides(bc_x, bc_y, sides):
    """Side kinds (left, right, bottom, top): `sides` if given, else bc_x twice, bc_y twice."""
    if sides is None:
        return (int(bc_x), int(bc_x), int(bc_y), int(bc_y))
    return tuple(int(k) for k in sides)


def _grid_sides(grid):
    """Side kinds and inflow states of an inputs.Grid."""
    kinds = grid.side_kinds() if hasattr(grid, "side_kinds") else \
        (grid.bc_x, grid.bc_x, grid.bc_y, grid.bc_y)
    inflow = {s: grid.inflow_state(s) for s in range(4)
              if hasattr(grid, "inflow_state") and grid.inflow_state(s) is not None}
    return kinds, inflow


class _Handle:
    """Calls shared by single-grid and batched handles."""

    h = None

    def _options(self, precision, linearisation, correction, limiter, graph_steps,
                 transonic=False, shock_limiter=False, flux_limiter=False):
        self.set_option(AF_OPT_PRECISION, precision)
        self.set_option(AF_OPT_LINEARISATION, linearisation)
        self.set_option(AF_OPT_CORRECTION, int(bool(correction)))
        self.set_option(AF_OPT_LIMITER, int(bool(limiter)))
        if graph_steps is not None:
            self.set_option(AF_OPT_GRAPH_STEPS, graph_steps)
        if transonic:
            self.set_option(AF_OPT_TRANSONIC, 1)
        if shock_limiter:
            self.set_option(AF_OPT_SHOCK_LIMITER, 1)
        if flux_limiter:
            self.set_option(AF_OPT_FLUX_LIMITER, 1)

    def _check(self, rc, create=False):
        if rc != AF_OK:
            msg = self.L.af_last_error(None if create else self.h)
            raise AfError(rc, (msg or b"").decode())

    def close(self):
        if self.h:
            self.L.af_destroy(self.h)
            self.h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key, value):
        self._check(self.L.af_set_option(self.h, key, int(value)))

    def get_option(self, key):
        v = ct.c_int64(0)
        self._check(self.L.af_get_option(self.h, key, ct.byref(v)))
        return v.value

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream (its .cuda_stream handle is used) or a raw handle."""
        handle = getattr(stream, "cuda_stream", stream)
        self._check(self.L.af_set_stream(self.h, ct.c_void_p(handle)))

    def step(self, dt):
        self._check(self.L.af_step(self.h, float(dt)))

    def run(self, t_end=float("inf"), cfl=0.3, max_steps=0):
        t = ct.c_double(0.0)
        n = ct.c_int64(0)
        self._check(self.L.af_run(self.h, float(t_end), float(cfl), int(max_steps),
                                  ct.byref(t), ct.byref(n)))
        return t.value, n.value

    def counters(self):
        c = (ct.c_int64 * AF_NCOUNTERS)()
        self._check(self.L.af_get_counters(self.h, c))
        return np.array(list(c), dtype=np.int64)

    def totals(self, g=0):
        """Domain totals of rho, rho u, rho v, E of grid g's current state (af_get_totals)."""
        o = np.zeros(4)
        self._check(self.L.af_get_totals(self.h, int(g), o.ctypes.data_as(_D)))
        return o

    def timing(self):
        """(ms in the point kernel, ms in the update kernel, steps) while timing is on."""
        o = (ct.c_double * 3)()
        self._check(self.L.af_get_timing(self.h, o))
        return o[0], o[1], int(o[2])

    def dof_count(self):
        return int(self.L.af_dof_count(self.h))

    def _set(self, g, shapes, avg, K, X, Y, t):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (avg, K, X, Y)]
        for a, (name, shp) in zip(arrs, shapes.items()):
            if a.shape != shp:
                raise ValueError(f"{name} has shape {a.shape}, expected {shp}")
        self._check(self.L.af_set_state_grid(self.h, g, *[_ptr(a) for a in arrs], float(t)))

    def _get(self, g, shapes):
        out = {k: np.empty(v, dtype=np.float64) for k, v in shapes.items()}
        t = ct.c_double(0.0)
        self._check(self.L.af_get_state_grid(self.h, g, _ptr(out["avg"]), _ptr(out["K"]),
                                             _ptr(out["X"]), _ptr(out["Y"]), ct.byref(t)))
        out["t"] = t.value
        return out

    def _set_inflow(self, g, side, W):
        w = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(4))
        self._check(self.L.af_set_inflow(self.h, int(g), int(side), _ptr(w)))

    def set_state_device(self, g, avg, K, X, Y, t=0.0):
        """State from device tensors (torch, FP64, contiguous, on the handle's GPU)."""
        shapes = self._shapes_of(g)
        arrs = (avg, K, X, Y)
        for a, (name, shp) in zip(arrs, shapes.items()):
            if tuple(a.shape) != shp or not a.is_contiguous() or str(a.dtype) != "torch.float64":
                raise ValueError(f"{name}: need a contiguous float64 tensor of shape {shp}")
        self._check(self.L.af_set_state_device(self.h, g, *[a.data_ptr() for a in arrs],
                                               float(t)))

    def get_state_device(self, g, avg, K, X, Y):
        """Copy the current state into device tensors (as for set_state_device); returns t."""
        shapes = self._shapes_of(g)
        for a, (name, shp) in zip((avg, K, X, Y), shapes.items()):
            if tuple(a.shape) != shp or not a.is_contiguous() or str(a.dtype) != "torch.float64":
                raise ValueError(f"{name}: need a contiguous float64 tensor of shape {shp}")
        t = ct.c_double(0.0)
        self._check(self.L.af_get_state_device(self.h, g, avg.data_ptr(), K.data_ptr(),
                                               X.data_ptr(), Y.data_ptr(), ct.byref(t)))
        return t.value

    def grid_info(self, g=0):
        """(t, steps taken) of grid g."""
        t = ct.c_double(0.0)
        n = ct.c_int64(0)
        self._check(self.L.af_get_grid_info(self.h, g, ct.byref(t), ct.byref(n)))
        return t.value, n.value


class Solver(_Handle):
    """One grid on the GPU.  Mirrors af_create / af_set_state / af_step / af_run / ..."""

    def __init__(self, nx, ny, x0, x1, y0, y1, gamma=1.4, bc_x=AF_BC_PERIODIC,
                 bc_y=AF_BC_PERIODIC, precision=AF_PREC_FP64, linearisation=AF_LIN_AF3,
                 correction=True, limiter=False, graph_steps=None, sides=None, inflow=None,
                 transonic=False, shock_limiter=False, flux_limiter=False):
        """sides: optional kinds (left, right, bottom, top) instead of bc_x / bc_y;
        inflow: optional {side: (rho, u, v, p)} for the inflow sides;
        transonic: Algorithm 2; shock_limiter: the shock-indicator blend (Sec. 3.4);
        flux_limiter: flux limiting of the cell averages (Sec. 3.5)."""
        self.L = load()
        self.nx, self.ny = int(nx), int(ny)
        k = _sides(bc_x, bc_y, sides)
        self.nkx = self.nx + (0 if k[0] == AF_BC_PERIODIC else 1)
        self.nky = self.ny + (0 if k[2] == AF_BC_PERIODIC else 1)
        self.h = _H()
        g = Grid(self.nx, self.ny, x0, x1, y0, y1)
        bc = Bc(*k)
        self._check(self.L.af_create(ct.byref(g), gamma, ct.byref(bc), ct.byref(self.h)),
                    create=True)
        self._options(precision, linearisation, correction, limiter, graph_steps, transonic,
                      shock_limiter, flux_limiter)
        for side, W in (inflow or {}).items():
            self.set_inflow(side, W)

    @classmethod
    def for_state(cls, st, **kw):
        g = st.grid
        kinds, inflow = _grid_sides(g)
        s = cls(g.nx, g.ny, g.x0, g.x1, g.y0, g.y1, st.gamma, sides=kinds, inflow=inflow, **kw)
        s.set_state(st.avg, st.K, st.X, st.Y, st.t)
        return s

    def set_inflow(self, side, W):
        self._set_inflow(0, side, W)

    def shapes(self):
        return _shapes(self.nx, self.ny, self.nkx, self.nky)

    def _shapes_of(self, g):
        return self.shapes()

    def set_state(self, avg, K, X, Y, t=0.0):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (avg, K, X, Y)]
        for a, (name, shp) in zip(arrs, self.shapes().items()):
            if a.shape != shp:
                raise ValueError(f"{name} has shape {a.shape}, expected {shp}")
        self._check(self.L.af_set_state(self.h, *[_ptr(a) for a in arrs], float(t)))

    def get_state(self):
        sh = self.shapes()
        out = {k: np.empty(v, dtype=np.float64) for k, v in sh.items()}
        t = ct.c_double(0.0)
        self._check(self.L.af_get_state(self.h, _ptr(out["avg"]), _ptr(out["K"]),
                                        _ptr(out["X"]), _ptr(out["Y"]), ct.byref(t)))
        out["t"] = t.value
        return out


class BatchSolver(_Handle):
    """Several independent grids in one handle (af_create_batch): one launch of each kernel
    per step for all grids, each grid with its own time step."""

    def __init__(self, grids, gamma=1.4, precision=AF_PREC_FP64, linearisation=AF_LIN_AF3,
                 correction=True, limiter=False, graph_steps=None, transonic=False,
                 shock_limiter=False):
        """grids: sequence of (nx, ny, x0, x1, y0, y1, bc_x, bc_y) or
        (nx, ny, x0, x1, y0, y1, (left, right, bottom, top))."""
        self.L = load()
        n = len(grids)
        G = (Grid * n)()
        B = (Bc * n)()
        self.dims = []
        for k, spec in enumerate(grids):
            nx, ny, x0, x1, y0, y1 = spec[:6]
            kinds = _sides(0, 0, spec[6]) if len(spec) == 7 else _sides(spec[6], spec[7], None)
            G[k] = Grid(int(nx), int(ny), x0, x1, y0, y1)
            B[k] = Bc(*kinds)
            self.dims.append((int(nx), int(ny),
                              int(nx) + (0 if kinds[0] == AF_BC_PERIODIC else 1),
                              int(ny) + (0 if kinds[2] == AF_BC_PERIODIC else 1)))
        self.h = _H()
        self._check(self.L.af_create_batch(n, G, gamma, B, ct.byref(self.h)), create=True)
        self._options(precision, linearisation, correction, limiter, graph_steps, transonic,
                      shock_limiter)

    @classmethod
    def for_states(cls, states, **kw):
        grids = [(st.grid.nx, st.grid.ny, st.grid.x0, st.grid.x1, st.grid.y0, st.grid.y1,
                  _grid_sides(st.grid)[0]) for st in states]
        s = cls(grids, states[0].gamma, **kw)
        for g, st in enumerate(states):
            for side, W in _grid_sides(st.grid)[1].items():
                s.set_inflow(g, side, W)
            s.set_state(g, st.avg, st.K, st.X, st.Y, st.t)
        return s

    def set_inflow(self, g, side, W):
        self._set_inflow(g, side, W)

    def __len__(self):
        return int(self.L.af_batch_size(self.h))

    def shapes(self, g):
        return _shapes(*self.dims[g])

    def _shapes_of(self, g):
        return self.shapes(g)

    def set_state(self, g, avg, K, X, Y, t=0.0):
        self._set(g, self.shapes(g), avg, K, X, Y, t)

    def get_state(self, g):
        return self._get(g, self.shapes(g))


def step_noalloc(grid, gamma, bc, ins, outs, pitch_avg, pitch_pts, dt, precision=AF_PREC_FP64,
                 linearisation=AF_LIN_AF3, correction=True, limiter=False, inflow=None,
                 stream=None):
    """af_step_noalloc: one step on caller-owned device arrays (addresses as ints, the
    library's device layout) with no allocation.  `grid`: (nx, ny, x0, x1, y0, y1); `bc`: side
    kinds (left, right, bottom, top); `ins`/`outs`: addresses of avg, K, X, Y; `inflow`: 4 x 4
    states or None.  Returns the step's counters; raises AfError on failure."""
    L = load()
    g = Grid(*grid)
    b = Bc(*bc)
    w = None
    if inflow is not None:
        w = np.ascontiguousarray(np.asarray(inflow, dtype=np.float64).reshape(16))
    cnt = (ct.c_int64 * AF_NCOUNTERS)()
    rc = L.af_step_noalloc(ct.byref(g), float(gamma), ct.byref(b),
                           w.ctypes.data_as(_D) if w is not None else None, int(precision),
                           int(linearisation), int(bool(correction)), int(bool(limiter)),
                           *[ct.c_void_p(int(p)) for p in ins], *[ct.c_void_p(int(p)) for p in outs],
                           int(pitch_avg), int(pitch_pts), float(dt),
                           ct.c_void_p(stream) if stream else None, cnt)
    if rc != 0:
        raise AfError(rc, L.af_last_error(None).decode())
    return list(cnt)
