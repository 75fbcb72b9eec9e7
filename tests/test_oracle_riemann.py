"""Pins of the exact Riemann solution used as the Sod-tube reference (Sec. III.C).

Checked against the textbook star state of Sod's problem (Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", Table 4.3, Test 1) and
against conditions any exact solution satisfies: the Rankine-Hugoniot jump
conditions across the shock and the Riemann invariant through the fan.
"""
import numpy as np
import pytest


def test_toro_test1_star_state(orc):
    _, _, _, ps, us = orc.riemann_exact(1.0, 1.0, 0.0, 0.125, 0.1, 0.0, 1.4, np.array([0.0]))
    assert ps == pytest.approx(0.30313, abs=1e-5)
    assert us == pytest.approx(0.92745, abs=1e-5)


@pytest.mark.parametrize("state", [(8.0, 10.0, 1.0, 1.0), (2.0, 10.0, 1.0, 1.0), (1.0, 1.0, 0.125, 0.1)])
def test_jump_and_fan_conditions(orc, state):
    rl, pl, rr, pr = state
    g = 2.0
    xi = np.linspace(-3, 3, 60001)
    rho, u, p, ps, us = orc.riemann_exact(rl, pl, 0.0, rr, pr, 0.0, g, xi)
    # shock on the right: locate it, then check the jump conditions
    cr = np.sqrt(g * pr / rr)
    S = cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    k = np.searchsorted(xi, S)
    r1, u1, p1 = rho[k - 3], u[k - 3], p[k - 3]
    E = lambda r, v, q: q / (g - 1) + 0.5 * r * v * v
    assert rr * (0 - S) == pytest.approx(r1 * (u1 - S), rel=1e-9)
    assert rr * 0 * (0 - S) + pr == pytest.approx(r1 * u1 * (u1 - S) + p1, rel=1e-9)
    assert E(rr, 0, pr) * (0 - S) + pr * 0 == pytest.approx(E(r1, u1, p1) * (u1 - S) + p1 * u1, rel=1e-9)
    # left rarefaction: u + 2c/(g-1) constant through the fan
    cl = np.sqrt(g * pl / rl)
    fan = (xi > -cl + 1e-3) & (xi < us - np.sqrt(g * ps / rho[np.searchsorted(xi, us) - 5]) - 1e-3)
    inv = u[fan] + 2 * np.sqrt(g * p[fan] / rho[fan]) / (g - 1)
    np.testing.assert_allclose(inv, 2 * cl / (g - 1), rtol=1e-10)
    # pressure and velocity continuous across the contact
    j = np.searchsorted(xi, us)
    assert p[j - 2] == pytest.approx(p[j + 2], rel=1e-12)
    assert u[j - 2] == pytest.approx(u[j + 2], rel=1e-12)
