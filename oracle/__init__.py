"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the plain FP64 CPU oracle (af_oracle.c).

Only tests/, the package smoke check and the CPU-baseline leg of bench.py may use this
module.  The oracle follows the paper (arXiv 2508.06273) step by step and shares no code
with the HIP library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MODE_AF3, MODE_AVG, MODE_SIMPLE = 0, 1, 2
KIND_K, KIND_X, KIND_Y = 0, 1, 2
OK, ERR_ARG, ERR_NONPHYSICAL, ERR_CFL = 0, -1, -2, -3
NCOUNTERS = 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over cells)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Cfg(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("x0", ct.c_double), ("y0", ct.c_double),
                ("dx", ct.c_double), ("dy", ct.c_double), ("gamma", ct.c_double),
                ("per_x", ct.c_int), ("per_y", ct.c_int), ("mode", ct.c_int),
                ("correction", ct.c_int), ("limiter", ct.c_int), ("gl_n", ct.c_int),
                ("nthreads", ct.c_int), ("bc", ct.c_int * 4), ("inflow", (ct.c_double * 4) * 4),
                ("tsw", ct.c_int), ("shock", ct.c_int), ("flux_limiter", ct.c_int)]


FIELD_CB = ct.CFUNCTYPE(None, ct.c_double, ct.c_double, ct.POINTER(ct.c_double))

_lib = None
_lock = threading.Lock()
_D = ct.POINTER(ct.c_double)
_LL = ct.POINTER(ct.c_longlong)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ct.CDLL(LIB)
            P = ct.POINTER(Cfg)
            L.or_step.argtypes = [P, _D, _D, _D, _D, ct.c_double, _LL]
            L.or_step.restype = ct.c_int
            L.or_max_speed.argtypes = [P, _D, _D, _D, _D]
            L.or_max_speed.restype = ct.c_double
            L.or_run.argtypes = [P, _D, _D, _D, _D, _D, ct.c_double, ct.c_double,
                                 ct.c_longlong, _LL, _LL]
            L.or_run.restype = ct.c_int
            L.or_gl.argtypes = [ct.c_int, _D, _D]
            L.or_p2c.argtypes = [_D, ct.c_double, _D]
            L.or_c2p.argtypes = [_D, ct.c_double, _D]
            L.or_corr.argtypes = [_D, _D, _D, ct.c_double, ct.c_double, _D]
            L.or_prep_cell.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, _D, _D]
            L.or_prep_cell.restype = ct.c_int
            L.or_eval_recon.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, ct.c_double,
                                        ct.c_double, _D]
            L.or_eval_recon.restype = ct.c_int
            L.or_dof_eg.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                    ct.c_int, _D, ct.c_double, _D]
            L.or_dof_eg.restype = ct.c_int
            L.or_dof_update.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, ct.c_int,
                                        ct.c_double, _D, _D, _LL]
            L.or_dof_update.restype = ct.c_int
            L.or_lf_point.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, ct.c_int,
                                      ct.c_double, _D]
            L.or_indicators.argtypes = [P, _D, _D, _D, _D, ct.c_int, ct.c_int, ct.c_int, _D,
                                        ct.POINTER(ct.c_int)]
            L.or_indicators.restype = ct.c_int
            L.or_lf_point.restype = ct.c_int
            L.or_eg_cb.argtypes = [ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.c_int, _D,
                                   ct.c_double, ct.c_double, FIELD_CB, ct.c_int, _D]
            L.or_eg_cb.restype = ct.c_int
            L.or_flux_theta.argtypes = [_D, _D, ct.c_double]
            L.or_flux_theta.restype = ct.c_double
            _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _v(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def cfg_for(state, mode=MODE_AF3, correction=True, limiter=False, gl_n=10, nthreads=0,
            tsw=False, shock=False, flux_limiter=False) -> Cfg:
    """tsw: Algorithm 2; shock: the shock-indicator blend of Sec. 3.4; flux_limiter: flux
    limiting of the cell averages (Sec. 3.5)."""
    g = state.grid
    c = Cfg(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, state.gamma, int(g.bc_x == 0),
            int(g.bc_y == 0), mode, int(correction), int(limiter), gl_n, nthreads)
    for s, k in enumerate(g.side_kinds()):
        c.bc[s] = k
        w = g.inflow_state(s)
        if w is not None:
            for v in range(4):
                c.inflow[s][v] = float(w[v])
    c.tsw = int(bool(tsw))
    c.shock = int(bool(shock))
    c.flux_limiter = int(bool(flux_limiter))
    return c


def _arrays(state):
    for name in ("avg", "K", "X", "Y"):
        a = getattr(state, name)
        if not (a.dtype == np.float64 and a.flags.c_contiguous):
            setattr(state, name, np.ascontiguousarray(a, dtype=np.float64))
    return state.avg, state.K, state.X, state.Y


def step(state, dt, **kw):
    """Advance `state` (in place) by one step of size dt. Returns (err, counters)."""
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    cnt = np.zeros(NCOUNTERS, dtype=np.int64)
    e = lib().or_step(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), float(dt),
                      cnt.ctypes.data_as(_LL))
    if e == OK:
        state.t += dt
    return e, cnt


def max_speed(state, **kw):
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    return lib().or_max_speed(ct.byref(c), _p(A), _p(K), _p(X), _p(Y))


def run(state, t_end, cfl, max_steps=0, **kw):
    """Advance `state` in place to t_end (or max_steps). Returns (err, steps, counters)."""
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    t = ct.c_double(state.t)
    n = ct.c_longlong(0)
    cnt = np.zeros(NCOUNTERS, dtype=np.int64)
    e = lib().or_run(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), ct.byref(t), float(t_end),
                     float(cfl), int(max_steps), ct.byref(n), cnt.ctypes.data_as(_LL))
    state.t = t.value
    return e, n.value, cnt


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().or_gl(n, _p(x), _p(w))
    return x, w


def p2c(U, gamma=1.4):
    U = _v(U)
    Q = np.zeros(4)
    lib().or_p2c(_p(U), gamma, _p(Q))
    return Q


def c2p(Q, gamma=1.4):
    Q = _v(Q)
    U = np.zeros(4)
    lib().or_c2p(_p(Q), gamma, _p(U))
    return U


def corr(U, Ux, Uy, tau, gamma=1.4):
    o = np.zeros(4)
    lib().or_corr(_p(_v(U)), _p(_v(Ux)), _p(_v(Uy)), gamma, tau, _p(o))
    return o


def prep_cell(state, i, j, **kw):
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    Uc = np.zeros(4)
    Ub = np.zeros(4)
    e = lib().or_prep_cell(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), i, j, _p(Uc), _p(Ub))
    return e, Uc, Ub


def eval_recon(state, i, j, x, y, **kw):
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    o = np.zeros(4)
    e = lib().or_eval_recon(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), i, j, x, y, _p(o))
    return e, o


def dof_eg(state, order, rec, kind, ci, cj, lin, tau, **kw):
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    o = np.zeros(4)
    e = lib().or_dof_eg(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), order, rec, kind, ci, cj,
                        _p(_v(lin)), float(tau), _p(o))
    return e, o


def dof_update(state, kind, ci, cj, dt, **kw):
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    h = np.zeros(4)
    f = np.zeros(4)
    cnt = np.zeros(NCOUNTERS, dtype=np.int64)
    e = lib().or_dof_update(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), kind, ci, cj, float(dt),
                            _p(h), _p(f), cnt.ctypes.data_as(_LL))
    return e, h, f, cnt


def lf_point(state, kind, ci, cj, tau, **kw):
    """Lax-Friedrichs point update of one DOF (the last branch of Algorithm 3)."""
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    o = np.zeros(4)
    e = lib().or_lf_point(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), kind, ci, cj, float(tau),
                          _p(o))
    return e, o


def indicators(state, kind, ci, cj, **kw):
    """(theta of Sec. 3.4, transonic flag of Algorithm 2) of one DOF from the state."""
    c = cfg_for(state, **kw)
    A, K, X, Y = _arrays(state)
    th = ct.c_double(0.0)
    f = ct.c_int(0)
    e = lib().or_indicators(ct.byref(c), _p(A), _p(K), _p(X), _p(Y), kind, ci, cj,
                            ct.byref(th), ct.byref(f))
    return e, th.value, f.value


def eg_field(order, xb, yb, vline, hline, lin, tau, field, gamma=1.4, gl_n=10):
    """Evolution operator applied to an analytic field(x, y) -> 4 primitive values."""
    def cb(x, y, out):
        v = field(x, y)
        for k in range(4):
            out[k] = float(v[k])
    f = FIELD_CB(cb)
    o = np.zeros(4)
    e = lib().or_eg_cb(order, xb, yb, int(vline), int(hline), _p(_v(lin)), float(tau), gamma,
                       f, gl_n, _p(o))
    return e, o


def flux_theta(Qlo, d, gamma=1.4):
    """Sec. 3.5: largest theta in [0, 1] with Qlo + theta d above the density/pressure floors."""
    return lib().or_flux_theta(_p(_v(Qlo)), _p(_v(d)), gamma)
