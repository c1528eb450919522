"""Test infrastructure: linear stability of the oracle's step about a uniform state.

The step is linearised by central differences of the oracle about a uniform state W0 on a
small periodic grid of unit cells: the response to a perturbation of each of the 16 degrees of
freedom of one cell (averages, K, X, Y; 4 variables each) gives the step's stencil, whose
Fourier transform is the amplification matrix G(k) of the mode exp(i (kx i + ky j)) (the step
commutes with shifts by whole cells).  The spectral radius of G(k), maximised over k, is the
growth factor per step of the linear scheme (paper Sec. 2; the CFL bound quoted there).

Run as a script it prints the spectral radius against the background Mach number and the CFL
number.
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_06273_amd import inputs as I  # noqa: E402

GAMMA = 1.4


def time_step(W0, cfl, gamma=GAMMA):
    """dt on unit cells for CFL number cfl: cfl / (max(|u|, |v|) + c) (paper Sec. 2)."""
    c = np.sqrt(gamma * W0[3] / W0[0])
    return cfl / (max(abs(W0[1]), abs(W0[2])) + c)


def impulse_response(W0, dt, n=8, eps=1e-6, gamma=GAMMA, **kw):
    """Oracle step linearised about W0: array (4 kinds, 4 vars, n, n, 16 inputs)."""
    g = I.Grid(n, n, 0.0, float(n), 0.0, float(n))
    base = I.uniform_state(g, W0, gamma)
    cols = []
    for kind in range(4):
        for v in range(4):
            outs = []
            for sgn in (1.0, -1.0):
                st = base.copy()
                arr = (st.avg, st.K, st.X, st.Y)[kind]
                arr[v, 0, 0] += sgn * eps
                e, _ = oracle.step(st, dt, **kw)
                if e != 0:
                    raise RuntimeError(f"oracle step failed: {e}")
                outs.append(np.stack([st.avg, st.K, st.X, st.Y]))
            cols.append((outs[0] - outs[1]) / (2.0 * eps))
    return np.stack(cols, axis=-1)


def amplification(R, k):
    """G(k) (16 x 16) from the impulse response R: sum over shifts s of R(s) exp(-i k.s)."""
    n = R.shape[2]
    s = np.arange(n)
    s = np.where(s >= n // 2, s - n, s)
    ph = np.exp(-1j * (k[0] * s[None, :] + k[1] * s[:, None]))  # [row j][column i]
    return np.einsum("abjic,ji->abc", R, ph).reshape(16, 16)


def spectral_radius(R, nk=33):
    """(max over a k grid on [-pi, pi]^2 of the spectral radius of G(k), the maximising k)."""
    best, kbest = -1.0, None
    for kx in np.linspace(-np.pi, np.pi, nk):
        for ky in np.linspace(-np.pi, np.pi, nk):
            r = float(np.abs(np.linalg.eigvals(amplification(R, (kx, ky)))).max())
            if r > best:
                best, kbest = r, (float(kx), float(ky))
    return best, kbest


def table(machs=(0.5, 0.7, 0.8, 0.85, 0.9, 0.95, 1.0, 1.05, 1.1, 1.2, 1.5),
          cfls=(0.1, 0.2, 0.279, 0.3)):
    """Rows: background (1, M c, 0, 1) and (1, M c, M c, 1); columns: CFL numbers."""
    c = np.sqrt(GAMMA)
    rows = []
    for diag in (False, True):
        for M in machs:
            u = M * c
            W0 = (1.0, u, u if diag else 0.0, 1.0)
            rows.append((W0, [spectral_radius(impulse_response(W0, time_step(W0, f)))[0]
                              for f in cfls]))
    return rows


if __name__ == "__main__":
    cfls = (0.1, 0.2, 0.279, 0.3)
    print("background (rho, u, v, p)      max(|u|,|v|)/c  " +
          "  ".join(f"CFL {f:<6}" for f in cfls))
    for W0, rs in table(cfls=cfls):
        M = max(abs(W0[1]), abs(W0[2])) / np.sqrt(GAMMA)
        print(f"({W0[0]:.2f}, {W0[1]:.3f}, {W0[2]:.3f}, {W0[3]:.2f})   {M:5.2f}        " +
              "  ".join(f"{r:.6f}" for r in rs), flush=True)
    W0 = (1.0, 1.0, 1.0, 1.0)
    for f in cfls:
        r, k = spectral_radius(impulse_response(W0, time_step(W0, f)))
        print(f"vortex background (1,1,1,1), CFL {f}: rho = {r:.6f} at k = ({k[0]:.3f}, {k[1]:.3f})")
