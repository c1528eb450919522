"""Test infrastructure: the Active Flux step linearised about a uniform state, in Fourier space.

This is an independent construction of the scheme of the paper (arXiv 2508.06273, Sec. 2) for
small perturbations of a uniform state W0 on a periodic grid of square cells (dx = dy = 1).  It
shares nothing with the oracle: the reconstruction is written as the nine-node Lagrange
interpolant, the circle integrals of eq. (EG2) are brute-force composite midpoint sums split
at the grid-line crossings (with Richardson extrapolation), and the unknowns are the Fourier
amplitudes of one cell's degrees of freedom.

About a uniform state the method is linear to first order: EG2 reproduces constants whatever
its linearisation state, so the dependence of Algorithm 1, the averaged and the simplified
linearisation on the data drops out, and the correction term of Corollary 1 is quadratic in
the derivatives.  One step then maps the amplitudes

    V = (A, K, X, Y)   A: conserved average, K/X/Y: primitive point values (4 each),

of the mode exp(i (kx i + ky j)) to G(k) V.  The layout of the sites follows the library and the
oracle: K(i, j) at (i, j), X(i, j) at (i, j + 1/2), Y(i, j) at (i + 1/2, j), cell (i, j) on
[i, i+1] x [j, j+1].
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def jac_p2c(W0, gamma=GAMMA):
    """dQ/dU of the ideal-gas map from primitive (rho, u, v, p) to conserved variables."""
    r, u, v, p = W0
    return np.array([[1, 0, 0, 0],
                     [u, r, 0, 0],
                     [v, 0, r, 0],
                     [0.5 * (u * u + v * v), r * u, r * v, 1 / (gamma - 1)]], float)


def jac_flux(W0, gamma=GAMMA):
    """df/dU and dg/dU (x and y fluxes of the Euler equations) with respect to (rho, u, v, p)."""
    r, u, v, p = W0
    H = gamma / (gamma - 1) * p / r + 0.5 * (u * u + v * v)  # total enthalpy
    # f = (r u, r u^2 + p, r u v, u (E + p)),  E + p = r (u^2 + v^2)/2 + gamma p/(gamma - 1)
    F = np.array([[u, r, 0, 0],
                  [u * u, 2 * r * u, 0, 1],
                  [u * v, r * v, r * u, 0],
                  [0.5 * u * (u * u + v * v), r * H + r * u * u, r * u * v,
                   gamma / (gamma - 1) * u]], float)
    G = np.array([[v, 0, r, 0],
                  [u * v, r * v, r * u, 0],
                  [v * v, 0, 2 * r * v, 1],
                  [0.5 * v * (u * u + v * v), r * u * v, r * H + r * v * v,
                   gamma / (gamma - 1) * v]], float)
    return F, G


def _lagrange(s):
    """Quadratic Lagrange basis on the nodes 0, 1/2, 1 at s (array)."""
    return np.stack([2 * (s - 0.5) * (s - 1), -4 * s * (s - 1), 2 * s * (s - 0.5)])


class Cell:
    """Fourier-amplitude reconstruction: cell (i, j) carries phase exp(i (kx i + ky j)) times the
    biquadratic of cell (0, 0), which interpolates the 8 boundary nodes and the centre value
    obtained by inverting the 2D Simpson rule in conserved variables."""

    def __init__(self, V, k, W0, gamma=GAMMA):
        kx, ky = k
        ex, ey = np.exp(1j * kx), np.exp(1j * ky)
        A, K, X, Y = V[0:4], V[4:8], V[8:12], V[12:16]
        T = jac_p2c(W0, gamma)
        nodes = np.zeros((3, 3, 4), complex)  # [a (x: 0, 1/2, 1)][b (y)][var]
        nodes[0, 0], nodes[2, 0], nodes[0, 2], nodes[2, 2] = K, ex * K, ey * K, ex * ey * K
        nodes[0, 1], nodes[2, 1] = X, ex * X
        nodes[1, 0], nodes[1, 2] = Y, ey * Y
        corners = nodes[0, 0] + nodes[2, 0] + nodes[0, 2] + nodes[2, 2]
        edges = nodes[0, 1] + nodes[2, 1] + nodes[1, 0] + nodes[1, 2]
        qc = (36 * A - T @ corners - 4 * (T @ edges)) / 16
        nodes[1, 1] = np.linalg.solve(T, qc)
        self.nodes = nodes
        self.k = (kx, ky)

    def __call__(self, x, y):
        """Values (4, n) at the points x, y (arrays of the same shape, any cells)."""
        ci, cj = np.floor(x), np.floor(y)
        lx, ly = _lagrange(x - ci), _lagrange(y - cj)
        val = np.einsum("an,bn,abv->vn", lx, ly, self.nodes)
        return val * np.exp(1j * (self.k[0] * ci + self.k[1] * cj))


def _circle_integrals(rec, xb, yb, W0, tau, n, gamma):
    """(1/pi) times the four circle integrals of eq. (EG2) and the foot-point value, by the
    composite midpoint rule with n nodes on each arc between crossings of the grid lines."""
    r0, u0, v0, p0 = W0
    c = np.sqrt(gamma * p0 / r0)
    px, py = xb - u0 * tau, yb - v0 * tau
    a = c * tau
    cuts = [0.0, 2 * np.pi]
    for line in np.arange(np.floor(px - a) - 1, np.ceil(px + a) + 2):  # x = line
        q = (line - px) / a
        if abs(q) < 1:
            t = np.arccos(q)
            cuts += [t, 2 * np.pi - t]
    for line in np.arange(np.floor(py - a) - 1, np.ceil(py + a) + 2):  # y = line
        q = (line - py) / a
        if abs(q) < 1:
            t = np.arcsin(q)
            cuts += [t % (2 * np.pi), (np.pi - t) % (2 * np.pi)]
    cuts = np.unique(np.array(cuts))
    th = []
    w = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        if hi - lo <= 0:
            continue
        m = (np.arange(n) + 0.5) / n
        th.append(lo + (hi - lo) * m)
        w.append(np.full(n, (hi - lo) / n))
    th = np.concatenate(th)
    w = np.concatenate(w)
    C, S = np.cos(th), np.sin(th)
    val = rec(px + a * C, py + a * S)  # (4, nodes)
    rho, u, v, p = val
    I_rho = np.sum(w * (p / c ** 2 - r0 / c * (u * C + v * S))) / np.pi
    I_u = np.sum(w * (-p * C / (r0 * c) + u * (2 * C * C - 0.5) + 2 * v * S * C)) / np.pi
    I_v = np.sum(w * (-p * S / (r0 * c) + 2 * u * S * C + v * (2 * S * S - 0.5))) / np.pi
    I_p = np.sum(w * (p - r0 * c * (u * C + v * S))) / np.pi
    foot = rec(np.array([px]), np.array([py]))[:, 0]
    return np.array([I_rho, I_u, I_v, I_p]), foot, c


def eg2(rec, xb, yb, W0, tau, n=2048, gamma=GAMMA):
    """EG2 (paper eq. EG2, linearised at W0) of the reconstruction `rec` at (xb, yb)."""
    def once(m):
        I, foot, c = _circle_integrals(rec, xb, yb, W0, tau, m, gamma)
        return np.array([foot[0] - 2 * foot[3] / c ** 2 + I[0], I[1], I[2], -foot[3] + I[3]])
    # midpoint error is O(1/n^2) on each smooth arc: one Richardson step
    return (4 * once(2 * n) - once(n)) / 3


SITES = {"K": (0.0, 0.0), "X": (0.0, 0.5), "Y": (0.5, 0.0)}


def step_matrix(W0, k, dt, n=2048, gamma=GAMMA):
    """G(k): the 16 x 16 amplification matrix of one step of size dt (cells of unit size)."""
    kx, ky = k
    Jq = jac_p2c(W0, gamma)
    Fj, Gj = jac_flux(W0, gamma)
    G = np.zeros((16, 16), complex)
    for col in range(16):
        V = np.zeros(16, complex)
        V[col] = 1.0
        rec = Cell(V, k, W0, gamma)
        new = {}
        half = {}
        for name, (xb, yb) in SITES.items():
            half[name] = eg2(rec, xb, yb, W0, 0.5 * dt, n, gamma)
            new[name] = eg2(rec, xb, yb, W0, dt, n, gamma)
        old = {"K": V[4:8], "X": V[8:12], "Y": V[12:16]}
        # Simpson in time (weights 1, 4, 1) and space on the west face (K(0,0), X(0,0), K(0,1))
        # and the south face (K(0,0), Y(0,0), K(1,0)); east / north faces carry the phase
        Fw = np.zeros(4, complex)
        Gs = np.zeros(4, complex)
        for wt, lvl in ((1, old), (4, half), (1, new)):
            Fw += wt * (Fj @ (lvl["K"] + 4 * lvl["X"] + np.exp(1j * ky) * lvl["K"]))
            Gs += wt * (Gj @ (lvl["K"] + 4 * lvl["Y"] + np.exp(1j * kx) * lvl["K"]))
        Fw /= 36.0
        Gs /= 36.0
        A_new = V[0:4] - dt * (np.exp(1j * kx) - 1) * Fw - dt * (np.exp(1j * ky) - 1) * Gs
        G[:, col] = np.concatenate([A_new, new["K"], new["X"], new["Y"]])
    assert Jq.shape == (4, 4)
    return G
