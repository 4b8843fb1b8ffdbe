"""Pins of the oracle's M4 kernel (section 2 of the paper names the M4 cubic
spline with support R = 2; its formula is the standard one of Monaghan &
Lattanzio 1985).

The properties checked here determine the kernel uniquely: a piecewise cubic
on [0, 2] with a knot at q = 1 that is even at the origin (f'(0) = 0), joins
zero at q = 2 with a triple root, is C2 at q = 1, and is normalised to unit
volume integral has exactly one free parameter left, fixed by normalisation.
A wrong coefficient, a dropped term or a wrong branch fails one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from conftest import read_golden

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def test_support_radius_matches_paper(orc):
    R = read_golden("paper_values.txt")["kernel_support_R_m4"]
    assert orc.kernel_f(R) == 0.0 and orc.kernel_df(R) == 0.0
    assert orc.kernel_f(R - 1e-6) > 0.0
    assert orc.kernel_f(3.7) == 0.0


def test_normalisation_unit_integral(orc):
    # 4 pi int_0^2h W(r,h) r^2 dr = 1 for any h
    for h in (0.3, 1.0, 2.5):
        f = lambda r: 4.0 * math.pi * r * r * orc.kernel_W(r, h)
        val = sum(integrate.quad(f, a * h, b * h, epsabs=1e-15, epsrel=1e-14)[0]
                  for a, b in ((0.0, 1.0), (1.0, 2.0)))
        assert abs(val - 1.0) < 1e-13


def test_dWdh_integrates_to_zero(orc):
    # d/dh of the unit normalisation vanishes
    for h in (0.5, 1.7):
        f = lambda r: 4.0 * math.pi * r * r * orc.kernel_dWdh(r, h)
        val = sum(integrate.quad(f, a * h, b * h, epsabs=1e-15, epsrel=1e-14)[0]
                  for a, b in ((0.0, 1.0), (1.0, 2.0)))
        assert abs(val) < 1e-12 / h ** 4


def test_even_at_origin_and_value(orc):
    assert orc.kernel_f(0.0) == 1.0
    assert orc.kernel_df(0.0) == 0.0
    eps = 1e-6
    assert abs(orc.kernel_f(eps) - orc.kernel_f(0.0)) < 1e-11


@pytest.mark.parametrize("q", [0.1, 0.5, 0.9, 1.1, 1.5, 1.9])
def test_df_is_derivative_of_f(orc, q):
    e = 1e-5
    fd = (orc.kernel_f(q + e) - orc.kernel_f(q - e)) / (2 * e)
    assert abs(fd - orc.kernel_df(q)) < 1e-9


def test_c2_continuity_at_knot(orc):
    e = 1e-7
    f_lo, f_hi = orc.kernel_f(1.0 - e), orc.kernel_f(1.0 + e)
    assert abs(f_lo - f_hi) < 1e-6
    d_lo, d_hi = orc.kernel_df(1.0 - e), orc.kernel_df(1.0 + e)
    assert abs(d_lo - d_hi) < 1e-6
    # second derivative from one-sided differences of df
    h = 1e-4
    dd_lo = (orc.kernel_df(1.0 - h) - orc.kernel_df(1.0 - 2 * h)) / h
    dd_hi = (orc.kernel_df(1.0 + 2 * h) - orc.kernel_df(1.0 + h)) / h
    assert abs(dd_lo - dd_hi) < 1e-3


def test_triple_root_at_support_edge(orc):
    # f ~ c (2 - q)^3 near q = 2: f / (2-q)^3 tends to a constant, df / (2-q)^2 too
    ratios = [orc.kernel_f(2.0 - t) / t ** 3 for t in (1e-2, 1e-3, 1e-4)]
    assert max(ratios) - min(ratios) < 1e-9
    dratios = [orc.kernel_df(2.0 - t) / t ** 2 for t in (1e-2, 1e-3, 1e-4)]
    assert max(dratios) - min(dratios) < 1e-9


def test_monotone_non_increasing(orc):
    qs = np.linspace(0.0, 2.2, 2001)
    f = np.array([orc.kernel_f(q) for q in qs])
    assert np.all(np.diff(f) <= 0.0)
    assert np.all(np.array([orc.kernel_df(q) for q in qs]) <= 0.0)


@pytest.mark.parametrize("r,h", [(0.3, 0.5), (0.7, 0.5), (0.95, 0.5), (1.2, 1.0)])
def test_gradient_and_h_derivative_by_finite_differences(orc, r, h):
    e = 1e-6
    fd_r = (orc.kernel_W(r + e, h) - orc.kernel_W(r - e, h)) / (2 * e)
    assert abs(fd_r - orc.kernel_dWdr(r, h)) < 1e-8 * max(1.0, abs(fd_r))
    fd_h = (orc.kernel_W(r, h + e) - orc.kernel_W(r, h - e)) / (2 * e)
    assert abs(fd_h - orc.kernel_dWdh(r, h)) < 1e-8 * max(1.0, abs(fd_h))


def test_scaling_with_h(orc):
    # W(r, h) = h^-3 W(r/h, 1): the kernel is a scaled shape function
    for q in (0.2, 0.8, 1.3, 1.8):
        for h in (0.01, 0.3, 4.0):
            assert orc.kernel_W(q * h, h) == pytest.approx(orc.kernel_W(q, 1.0) / h ** 3, rel=1e-14)
