"""Pins of the exact Riemann solver that the rarefaction tests compare with
(tests/exact_riemann.py): printed textbook values, the jump conditions across a shock, the
Riemann invariant across a fan, and the vacuum case."""
import math

import numpy as np

import exact_riemann as ER

G = 1.4


def test_sod_star_state_matches_the_textbook():
    """Sod's problem (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1): star pressure 0.30313, star
    velocity 0.92745, star densities 0.42632 (left) and 0.26557 (right), as tabulated by Toro
    (Riemann Solvers and Numerical Methods for Fluid Dynamics, Table 4.3, test 1)."""
    WL, WR = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1)
    p, u = ER.star_state(WL, WR, G)
    assert abs(p - 0.30313) < 1e-5 and abs(u - 0.92745) < 1e-5
    left_star = ER.sample(WL, WR, u - 1e-6, G)
    right_star = ER.sample(WL, WR, u + 1e-6, G)
    assert abs(left_star[0] - 0.42632) < 1e-5 and abs(right_star[0] - 0.26557) < 1e-5


def _cons_flux(W):
    r, u, v, p = W
    E = p / (G - 1) + 0.5 * r * (u * u + v * v)
    return np.array([r, r * u, E]), np.array([r * u, r * u * u + p, u * (E + p)])


def test_shock_satisfies_the_jump_conditions():
    """The right-moving shock of Sod's problem: with S = (m2 - m1) / (q2 - q1) from the mass
    equation, momentum and energy satisfy F2 - F1 = S (Q2 - Q1) too."""
    WL, WR = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1)
    p, u = ER.star_state(WL, WR, G)
    pre = ER.sample(WL, WR, 10.0, G)          # ahead of the shock
    post = ER.sample(WL, WR, u + 1e-9, G)     # behind it, in the star region
    Q1, F1 = _cons_flux(pre)
    Q2, F2 = _cons_flux(post)
    S = (F2[0] - F1[0]) / (Q2[0] - Q1[0])
    assert np.allclose(F2 - F1, S * (Q2 - Q1), rtol=1e-10, atol=1e-12)
    assert S > u  # the shock runs ahead of the contact


def test_fan_keeps_its_riemann_invariant():
    """Across a left rarefaction u + 2c/(gamma - 1) is constant and the entropy p / rho^gamma
    too (the transonic rarefaction of the paper's test, right fan: u - 2c/(gamma - 1))."""
    WL, WR = (0.1, -2.0, 0.0, 0.1), (1.0, -1.0, 0.0, 1.0)
    p, u = ER.star_state(WL, WR, G)
    assert p < WR[3]  # the right wave is a rarefaction
    inv, ent = [], []
    for s in np.linspace(u + 0.05, WR[1] + math.sqrt(G * WR[3] / WR[0]) - 0.05, 25):
        r, uu, _, pp = ER.sample(WL, WR, s, G)
        c = math.sqrt(G * pp / r)
        inv.append(uu - 2 * c / (G - 1))
        ent.append(pp / r ** G)
    assert np.ptp(inv) < 1e-12 and np.ptp(ent) < 1e-12
    # the fan is transonic: inside it u + c = x/t, negative at its tail, positive at its head
    for s in (-0.5, 0.1):
        w = ER.sample(WL, WR, s, G)
        assert abs(w[1] + math.sqrt(G * w[3] / w[0]) - s) < 1e-12


def test_double_rarefaction_opens_a_vacuum():
    """(7, -1, 0.2) | (7, 1, 0.2): u_R - u_L = 2 = 2 (c_L + c_R) / (gamma - 1) with c = 0.2, the
    threshold at which the fans separate: vacuum at x/t = 0, where both fans' tails end."""
    WL, WR = (7.0, -1.0, 0.0, 0.2), (7.0, 1.0, 0.0, 0.2)
    assert ER.star_state(WL, WR, G) is None
    mid = ER.sample(WL, WR, 0.0, G)
    assert mid[0] < 1e-12 and mid[3] < 1e-12  # the fans' tails meet at x/t = 0 up to rounding
    # symmetry: rho even, u odd in x/t
    for s in (0.3, 0.7, 1.1):
        a, b = ER.sample(WL, WR, s, G), ER.sample(WL, WR, -s, G)
        assert abs(a[0] - b[0]) < 1e-13 and abs(a[1] + b[1]) < 1e-13
    # mass balance on [0, 1]: the undisturbed states carry rho |u| = 7 out through both ends
    # (the fans' heads, at speed 1.2, stay inside until t = 5/12), so at t = 0.3 the mass is
    # 7 - 2 * 7 * 0.3
    avg = ER.cell_averages(WL, WR, 0.5, 0.3, np.linspace(0.0, 1.0, 65), G, sub=64)
    assert abs(avg[0].mean() - (7.0 - 2 * 7.0 * 0.3)) < 2e-3
