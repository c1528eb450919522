"""Steady oblique shock relations of the ideal gas (Rankine-Hugoniot across a straight shock
at angle beta to the upstream flow): the exact states of the regular shock reflection."""
import math

import numpy as np
from scipy.optimize import brentq


def across_shock(W, beta, gamma=1.4):
    """Primitive state behind a straight shock inclined at beta (radians, measured from the
    upstream flow direction, turning the flow towards the shock) to the state W."""
    rho, u, v, p = W
    V = math.hypot(u, v)
    phi = math.atan2(v, u)
    c = math.sqrt(gamma * p / rho)
    Mn = V * math.sin(beta) / c
    r = (gamma + 1) * Mn ** 2 / ((gamma - 1) * Mn ** 2 + 2)
    p2 = p * (1 + 2 * gamma / (gamma + 1) * (Mn ** 2 - 1))
    vt = V * math.cos(beta)
    vn = V * math.sin(beta) / r
    return rho * r, vt, vn, p2, phi


def deflection(W, beta, gamma=1.4):
    """Flow turning angle of a shock at beta."""
    _, vt, vn, _, _ = across_shock(W, beta, gamma)
    V = math.hypot(W[1], W[2])
    return beta - math.atan2(vn, vt) if V > 0 else 0.0


def turned_state(W, beta, sign, gamma=1.4):
    """State behind the shock; the flow turns by the deflection angle with sign `sign`
    (+1: counter-clockwise) relative to the upstream direction."""
    rho2, vt, vn, p2, phi = across_shock(W, beta, gamma)
    V2 = math.hypot(vt, vn)
    th = beta - math.atan2(vn, vt)
    ang = phi + sign * th
    return np.array([rho2, V2 * math.cos(ang), V2 * math.sin(ang), p2])


def weak_shock_angle(W, theta, gamma=1.4):
    """Weak-solution shock angle that turns the flow by theta (radians, > 0)."""
    rho, u, v, p = W
    M = math.hypot(u, v) / math.sqrt(gamma * p / rho)
    mu = math.asin(1.0 / M)
    # the deflection grows from 0 at the Mach angle to its maximum, then falls
    bs = np.linspace(mu + 1e-9, 0.5 * math.pi - 1e-9, 2001)
    d = [deflection(W, b, gamma) for b in bs]
    k = int(np.argmax(d))
    if d[k] < theta:
        raise ValueError("deflection beyond the attached-shock limit")
    return brentq(lambda b: deflection(W, b, gamma) - theta, bs[0], bs[k], xtol=1e-15)
