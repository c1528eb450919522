"""The oracle's whole step about a uniform state, against an independent linear construction.

About a uniform state the step is linear to first order (EG2 reproduces constants whatever its
linearisation state; the correction of Corollary 1 is quadratic in the derivatives).  The
oracle's step, linearised by central differences (tests/stability.py), must then equal the
Fourier-space construction of the paper's linear scheme in tests/linear_af.py, which builds the
nine-node reconstruction, eq. (EG2) by brute-force arc sums and the Simpson fluxes of eqs. (F)
and (2dfvm) with no code in common with the oracle.  A dropped term, a wrong sign or index, or
a transposed operand anywhere in the oracle's step shows up in one of the 256 entries of some
G(k).

The same amplification matrices decide linear stability (paper Sec. 2 quotes stability of the
linear EG2 Active Flux schemes for CFL <= 0.279).  They show the scheme stable for background
flows below Mach 0.8 along the axes and above Mach 1, and unstable in between, at every CFL
number: the background (1, 1, 1, 1) of the isentropic vortex (Mach 0.845 along each axis)
grows by 0.6 % per step at CFL 0.279.
"""
import numpy as np
import pytest

import linear_af as L
import stability as S

# backgrounds with non-zero velocities: about a zero velocity the foot point of EG2 sits on a
# grid line, where the one-sided derivatives of the reconstruction differ; the step is still
# differentiable there, but its central differences carry an O(eps) term
BACKGROUNDS = [(1.0, 1.0, 1.0, 1.0), (1.0, 1.1, 0.3, 1.0), (1.2, -0.4, 0.7, 0.8),
               (0.9, 0.2, -1.5, 1.3)]
KS = [(0.0, 0.0), (-0.589, -0.589), (1.3, -0.4), (np.pi, 2.0)]


@pytest.mark.parametrize("W0", BACKGROUNDS)
@pytest.mark.parametrize("opts", [dict(mode=0, correction=True), dict(mode=2, correction=False),
                                  dict(mode=1, correction=True)])
def test_linearised_step_matches_independent_construction(W0, opts):
    dt = S.time_step(W0, 0.279)
    R = S.impulse_response(W0, dt, **opts)
    for k in KS:
        Go = S.amplification(R, k)
        Gl = L.step_matrix(W0, k, dt, n=1024)
        assert np.abs(Go - Gl).max() < 2e-8, (W0, k, np.abs(Go - Gl).max())


def test_linear_construction_is_consistent():
    """Self-check of the independent construction: a uniform perturbation (k = 0, all DOFs
    equal in primitive variables, the average its conserved image) is preserved, up to the
    error of its arc sums."""
    W0 = (1.0, 0.6, -0.3, 1.0)
    dt = S.time_step(W0, 0.2)
    G0 = L.step_matrix(W0, (0.0, 0.0), dt, n=512)
    dU = np.array([0.3, -0.2, 0.5, 0.7])
    V = np.concatenate([L.jac_p2c(W0) @ dU, dU, dU, dU])
    assert np.abs(G0 @ V - V).max() < 1e-10


def test_stability_map_of_the_scheme():
    """Spectral radius of G(k) over k: 1 (to rounding) where the paper's bound applies and the
    flow is well below or above sonic along the axes; above 1 for near-sonic backgrounds at
    every CFL number, the isentropic-vortex background included."""
    stable = [(1.0, 0.0, 0.0, 1.0), (1.0, 0.5, 0.5, 1.0), (1.0, 0.9, 0.0, 1.0), (1.0, 2.0, 2.0, 1.0),
              (1.2, -0.4, 0.7, 0.8)]
    for W0 in stable:
        r, _ = S.spectral_radius(S.impulse_response(W0, S.time_step(W0, 0.279)), nk=17)
        assert r < 1.0 + 1e-7, (W0, r)
    vortex = (1.0, 1.0, 1.0, 1.0)
    grow = {}
    for cfl in (0.1, 0.279):
        grow[cfl], _ = S.spectral_radius(S.impulse_response(vortex, S.time_step(vortex, cfl)),
                                         nk=33)
    assert grow[0.1] > 1.001 and grow[0.279] > 1.005
    # growth per unit time t (steps per unit time ~ 1 / CFL) hardly depends on the CFL number
    rate = {f: np.log(g) / f for f, g in grow.items()}
    assert 0.5 < rate[0.1] / rate[0.279] < 1.0
