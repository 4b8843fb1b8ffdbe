"""Pins of the oracle's quintic spline kernel (section 2 names it, with
support R = 3, after Morris 1996) and of every sum run with it.

* Shape: f(0) = 66, f(1) = 26, f(2) = 1, f(q >= 3) = 0 and f'(0) = 0 from
  the B-spline form; the piecewise quintic is C^4, so f and its first four
  derivatives (by finite differences of the oracle's f) join at the knots
  q = 1 and 2; the oracle's f' equals a central difference of its f.
* Normalisation: 4 pi sigma int_0^3 f(q) q^2 dq = 1 with sigma = 1/(120 pi),
  by adaptive quadrature of the oracle's own f; and on a perfect periodic
  lattice the density sum at h = 1.2 spacings equals the mean density to
  1e-5 (the quintic's lattice sum error is far below the M4's).
* The density solve: h = eta (m/rho)^(1/3) holds at the root, drho/dh equals
  a central difference of the density sum in h, and the neighbour count
  equals a numpy brute-force count of 0 < r < 3h.
* Forces: the support is 3 max(h_i, h_j) in the force loop too -- the force
  neighbour count equals a brute-force count, and on a perfect lattice the
  grad-h velocity divergence of a linear field is exact, which needs the
  force loop and drho/dh to share the kernel and its support.
* Momentum and energy are conserved to roundoff on a jittered set with
  viscosity, and the sampled one-by-one evaluation equals the O(N^2) one.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1709_04488_amd import workloads as W


def test_shape_values(orc):
    assert orc.quintic_f(0.0) == 66.0
    assert orc.quintic_f(1.0) == 26.0
    assert orc.quintic_f(2.0) == 1.0
    assert orc.quintic_f(3.0) == 0.0 and orc.quintic_f(3.5) == 0.0
    assert orc.quintic_df(0.0) == 0.0
    assert orc.quintic_df(3.0) == 0.0
    # monotone decreasing on (0, 3)
    q = np.linspace(0.01, 2.99, 300)
    f = np.array([orc.quintic_f(v) for v in q])
    assert np.all(np.diff(f) < 0.0)
    assert np.all(np.array([orc.quintic_df(v) for v in q]) < 0.0)


def test_derivative_is_the_slope_of_f(orc):
    eps = 1e-6
    for q in (0.05, 0.4, 0.999, 1.3, 1.75, 2.2, 2.9):
        fd = (orc.quintic_f(q + eps) - orc.quintic_f(q - eps)) / (2 * eps)
        assert orc.quintic_df(q) == pytest.approx(fd, rel=1e-7, abs=1e-7)


@pytest.mark.parametrize("knot", [1.0, 2.0])
def test_smooth_at_the_knots(orc, knot):
    """Derivatives 0..4 from the left and the right agree at each knot
    (one-sided finite-difference stencils of the oracle's f)."""
    e = 1e-3
    f = orc.quintic_f

    def left(k):
        pts = [f(knot - j * e) for j in range(6)]
        # backward differences: k-th derivative ~ nabla^k f / e^k
        d = np.array(pts)
        for _ in range(k):
            d = d[:-1] - d[1:]
        return d[0] / e ** k

    def right(k):
        pts = [f(knot + j * e) for j in range(6)]
        d = np.array(pts)
        for _ in range(k):
            d = d[1:] - d[:-1]
        return d[0] / e ** k

    for k in range(4):
        a, b = left(k), right(k)
        # one-sided stencils carry O(e) error in each derivative
        assert a == pytest.approx(b, rel=0.02, abs=0.6 * 10 ** k * e * 100), (knot, k)
    # the fifth derivative jumps (a piecewise quintic is C^4, not C^5)


def test_normalisation(orc):
    val, err = integrate.quad(lambda q: orc.quintic_f(q) * q * q, 0.0, 3.0, points=[1.0, 2.0],
                              epsabs=1e-13, epsrel=1e-13)
    assert val == pytest.approx(30.0, rel=1e-12)        # 1 / (4 pi sigma), sigma = 1/(120 pi)
    # sigma used by the sums: on a lattice the kernel sum equals the integral
    w = W.lattice(10)
    a = w.arrays
    p = orc.Params(**w.setup, kernel=orc.KERNEL_QUINTIC)
    rho0 = np.sum(a["m"])                              # unit box
    sel = np.array([0, 123, 777])
    r = orc.rho_at(p, a["x"], a["y"], a["z"], a["m"], np.full(3, 0.12), sel=sel)
    assert np.allclose(r["rho"], rho0, rtol=1e-5)
    # the M4 with the same h misses by far more (its lattice error is larger)
    m4 = orc.rho_at(orc.Params(**w.setup), a["x"], a["y"], a["z"], a["m"], np.full(3, 0.12),
                    sel=sel)
    assert np.all(np.abs(m4["rho"] / rho0 - 1.0) > 10 * np.abs(r["rho"] / rho0 - 1.0))


def test_density_solve(orc):
    w = W.jittered_lattice(8, seed=21)
    a = w.arrays
    p = orc.Params(**w.setup, kernel=orc.KERNEL_QUINTIC)
    d = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])
    assert np.allclose(d["h"], 1.2 * (a["m"] / d["rho"]) ** (1.0 / 3.0), rtol=1e-10)
    sel = np.array([3, 99, 400])
    eps = 1e-6
    hs = d["h"][sel]
    up = orc.rho_at(p, a["x"], a["y"], a["z"], a["m"], hs * (1 + eps), sel=sel)
    dn = orc.rho_at(p, a["x"], a["y"], a["z"], a["m"], hs * (1 - eps), sel=sel)
    fd = (up["rho"] - dn["rho"]) / (2 * eps * hs)
    assert np.allclose(d["drhodh"][sel], fd, rtol=1e-6)
    # neighbour count (self excluded): brute force r < 3h over the minimum image
    for k, i in enumerate(sel.tolist()):
        dd = np.stack([a["x"] - a["x"][i], a["y"] - a["y"][i], a["z"] - a["z"][i]])
        dd -= np.round(dd)
        r = np.sqrt(np.sum(dd * dd, axis=0))
        assert d["nngb"][i] == np.sum(r < 3.0 * d["h"][i]) - 1
    # about (4/3) pi (3 eta)^3 = 195 neighbours, 3.4 times the M4's 58
    assert abs(np.mean(d["nngb"]) - 4.0 / 3.0 * math.pi * 3.6 ** 3) < 6


def _lattice_open(n_side):
    k = np.arange(n_side, dtype=np.float64)
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def test_force_support_and_exact_divergence(orc):
    x, y, z = _lattice_open(17)
    n = x.size
    A = np.random.default_rng(9).normal(0, 1, (3, 3))
    pos = np.stack([x, y, z])
    v = A @ pos
    m = np.ones(n)
    p = orc.Params(periodic=False, kernel=orc.KERNEL_QUINTIC)
    d = orc.density(p, x, y, z, m, np.full(n, 1.2))
    f = orc.forces(p, x, y, z, v[0], v[1], v[2], m, np.ones(n), d["h"], d["rho"], d["omega"])
    reach = 3.0 * d["h"].max() + 1.0
    inner = np.all(np.abs(pos - 8.0) <= 8.0 - reach, axis=0)
    assert inner.sum() >= 1
    curl = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    assert np.max(np.abs(f["divv"][inner] - np.trace(A))) < 1e-12 * np.abs(A).sum()
    assert np.max(np.abs(f["curlv"][inner] - np.linalg.norm(curl))) < 1e-12 * np.abs(A).sum()
    for i in np.nonzero(inner)[0][:3].tolist() + [0, n - 1]:
        r = np.sqrt((x - x[i]) ** 2 + (y - y[i]) ** 2 + (z - z[i]) ** 2)
        cnt = np.sum((r < 3.0 * d["h"][i]) | (r < 3.0 * d["h"])) - 1     # self excluded
        assert f["nforce"][i] == cnt


def test_conservation_and_sampled_evaluation(orc):
    w = W.jittered_lattice(8, seed=23, sigma_v=0.2)
    a = w.arrays
    p = orc.Params(**w.setup, kernel=orc.KERNEL_QUINTIC)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    m = a["m"]
    mom = [np.sum(m * ev[k]) for k in ("ax", "ay", "az")]
    assert max(abs(q) for q in mom) < 1e-13 * np.sum(m * ev["scale_a"])
    e = np.sum(m * (a["vx"] * ev["ax"] + a["vy"] * ev["ay"] + a["vz"] * ev["az"] + ev["dudt"]))
    scale = np.sum(m * (ev["scale_a"] * np.sqrt(a["vx"] ** 2 + a["vy"] ** 2 + a["vz"] ** 2)
                        + ev["scale_u"]))
    assert abs(e) < 1e-13 * scale
    sel = np.array([0, 77, 300, 511])
    s = orc.sampled_evaluation(p, a, sel)
    for k in ("h", "rho", "omega"):
        assert np.allclose(s.values[k], ev[k][sel], rtol=1e-12), k
    for k in ("ax", "ay", "az", "dudt"):
        sk = "scale_u" if k == "dudt" else "scale_a"
        assert np.max(np.abs(s.values[k] - ev[k][sel]) / ev[sk][sel]) < 1e-12, k
    assert np.array_equal(s.n_force, ev["nforce"][sel])
