"""Pins of the oracle's equation of state (orc_eos).

Section 2.1.1 gives the ideal-gas pressure P = (gamma - 1) rho u.  The sound
speed is not printed; the reading taken is the adiabatic one,
c^2 = (dP/drho) at constant entropy = gamma P / rho.  Both are pinned here
by values worked by hand and by a derivative taken along an adiabat, which
does not use the formula for c at all.
"""
import math

import numpy as np
import pytest


def test_hand_worked_values(orc):
    # rho = 2, u = 3, gamma = 5/3: P = (2/3) * 2 * 3 = 4,
    # c = sqrt((5/3) * 4 / 2) = sqrt(10/3)
    P, c = orc.eos(5.0 / 3.0, [2.0], [3.0])
    assert P[0] == pytest.approx(4.0, rel=1e-15)
    assert c[0] == pytest.approx(math.sqrt(10.0 / 3.0), rel=1e-15)
    # gamma = 1.4, rho = 0.5, u = 2.5: P = 0.4 * 0.5 * 2.5 = 0.5,
    # c^2 = 1.4 * 0.5 / 0.5 = 1.4
    P, c = orc.eos(1.4, [0.5], [2.5])
    assert P[0] == pytest.approx(0.5, rel=1e-15)
    assert c[0] == pytest.approx(math.sqrt(1.4), rel=1e-15)


def test_sound_speed_is_the_adiabatic_derivative(orc):
    """Along an adiabat du = (P / rho^2) drho (first law, no heat); then
    u = u0 (rho / rho0)^(gamma - 1) and P(rho) = (gamma - 1) rho u(rho).  The
    sound speed squared must equal dP/drho there, taken here by a central
    difference of P along that curve (no use of gamma P / rho)."""
    rng = np.random.default_rng(4)
    for gamma in (5.0 / 3.0, 1.4, 1.1):
        rho0 = rng.uniform(0.1, 10.0, 16)
        u0 = rng.uniform(0.1, 10.0, 16)
        P0, c = orc.eos(gamma, rho0, u0)
        d = 1e-4 * rho0
        up = u0 * ((rho0 + d) / rho0) ** (gamma - 1.0)
        um = u0 * ((rho0 - d) / rho0) ** (gamma - 1.0)
        Pp, _ = orc.eos(gamma, rho0 + d, up)
        Pm, _ = orc.eos(gamma, rho0 - d, um)
        dPdrho = (Pp - Pm) / (2.0 * d)
        assert np.max(np.abs(c ** 2 / dPdrho - 1.0)) < 1e-7, gamma
        # and the pressure is linear in rho u with slope gamma - 1
        assert np.allclose(P0, (gamma - 1.0) * rho0 * u0, rtol=1e-15, atol=0.0)


def test_sound_speed_depends_on_u_only(orc):
    # c^2 = gamma (gamma - 1) u: the same u at any density gives the same c
    P, c = orc.eos(5.0 / 3.0, [1e-3, 1.0, 1e3], [0.7, 0.7, 0.7])
    assert np.allclose(c, math.sqrt(5.0 / 3.0 * 2.0 / 3.0 * 0.7), rtol=1e-15)
    assert P[2] / P[0] == pytest.approx(1e6, rel=1e-14)
