"""Exact solution of the Riemann problem of the 1D Euler equations for an ideal gas, after the
textbook construction of E. F. Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
ch. 4: the star pressure is the root of f(p) = f_L(p) + f_R(p) + u_R - u_L, where f_K is the
shock (p > p_K) or rarefaction (p <= p_K) branch; the solution at x/t is then sampled across
the left wave, the contact and the right wave.  When the two rarefactions cannot meet
(u_R - u_L >= 2 (c_L + c_R) / (gamma - 1)) a vacuum opens between them.

Used by the tests as an independent reference; it shares nothing with the oracle or the
library."""
import math

import numpy as np
from scipy.optimize import brentq


def _f(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(WL, WR, gamma=1.4):
    """(p*, u*) of the Riemann problem, or None if a vacuum opens."""
    rl, ul, _, pl = WL
    rr, ur, _, pr = WR
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    # the fans separate (a vacuum opens) once u_R - u_L reaches 2 (c_L + c_R) / (gamma - 1);
    # data set exactly at that threshold hit it only up to the rounding of c
    if ur - ul >= 2.0 * (cl + cr) / (gamma - 1.0) * (1.0 - 1e-12):
        return None
    g = lambda p: _f(p, rl, pl, gamma) + _f(p, rr, pr, gamma) + ur - ul
    hi = max(pl, pr)
    while g(hi) < 0.0:
        hi *= 2.0
    p = brentq(g, 1e-300, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    u = 0.5 * (ul + ur) + 0.5 * (_f(p, rr, pr, gamma) - _f(p, rl, pl, gamma))
    return p, u


def _rarefaction_inside(W, s, gamma, left):
    """State inside a rarefaction fan at speed s (left or right facing)."""
    rho, u, _, p = W
    c = math.sqrt(gamma * p / rho)
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), 2.0 / (gamma + 1.0)
    if left:
        cf = g2 * c + g1 * (u - s)
        uf = g2 * (c + 0.5 * (gamma - 1.0) * u + s)
    else:
        cf = g2 * c - g1 * (u - s)
        uf = g2 * (-c + 0.5 * (gamma - 1.0) * u + s)
    rf = rho * (cf / c) ** (2.0 / (gamma - 1.0))
    pf = p * (cf / c) ** (2.0 * gamma / (gamma - 1.0))
    return rf, uf, pf


def sample(WL, WR, s, gamma=1.4):
    """Primitive (rho, u, v, p) at x/t = s; v is carried by the contact."""
    rl, ul, vl, pl = WL
    rr, ur, vr, pr = WR
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    star = star_state(WL, WR, gamma)
    if star is None:  # two rarefactions with a vacuum between them
        sl_head, sr_head = ul - cl, ur + cr
        sl_tail = ul + 2.0 * cl / (gamma - 1.0)
        sr_tail = ur - 2.0 * cr / (gamma - 1.0)
        if s <= sl_head:
            return np.array([rl, ul, vl, pl])
        if s >= sr_head:
            return np.array([rr, ur, vr, pr])
        if s < sl_tail:
            r, u, p = _rarefaction_inside(WL, s, gamma, True)
            return np.array([r, u, vl, p])
        if s > sr_tail:
            r, u, p = _rarefaction_inside(WR, s, gamma, False)
            return np.array([r, u, vr, p])
        return np.array([0.0, s, 0.5 * (vl + vr), 0.0])
    ps, us = star
    g = gamma
    if s <= us:  # left of the contact
        if ps > pl:  # left shock
            sh = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sh:
                return np.array([rl, ul, vl, pl])
            r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
            return np.array([r, us, vl, ps])
        cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
        if s <= ul - cl:
            return np.array([rl, ul, vl, pl])
        if s >= us - cs:
            return np.array([rl * (ps / pl) ** (1 / g), us, vl, ps])
        r, u, p = _rarefaction_inside(WL, s, g, True)
        return np.array([r, u, vl, p])
    if ps > pr:  # right shock
        sh = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sh:
            return np.array([rr, ur, vr, pr])
        r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
        return np.array([r, us, vr, ps])
    cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
    if s >= ur + cr:
        return np.array([rr, ur, vr, pr])
    if s <= us + cs:
        return np.array([rr * (ps / pr) ** (1 / g), us, vr, ps])
    r, u, p = _rarefaction_inside(WR, s, g, False)
    return np.array([r, u, vr, p])


def cell_averages(WL, WR, x0, t, edges, gamma=1.4, sub=64):
    """Conserved cell averages (rho, rho u, rho v, E) of the exact solution at time t on the
    cells [edges[i], edges[i+1]], by the midpoint rule on `sub` sub-intervals per cell."""
    n = len(edges) - 1
    out = np.zeros((4, n))
    for i in range(n):
        xs = edges[i] + (np.arange(sub) + 0.5) / sub * (edges[i + 1] - edges[i])
        acc = np.zeros(4)
        for x in xs:
            r, u, v, p = sample(WL, WR, (x - x0) / t, gamma)
            acc += [r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v)]
        out[:, i] = acc / sub
    return out
