"""Pins of the oracle's density loop and h-rho solve (eqs. EQN:SPHRHO,
EQN:HRHO, EQN:OMEGA) against things fixed outside the oracle: an
independent high-precision lattice sum, a closed-form few-body case, a
library neighbour search, the paper's <1 % density-offset statement, the
h-rho relation itself and finite differences."""
import mpmath as mp
import numpy as np
import pytest
from scipy.spatial import cKDTree

from conftest import read_golden
from paper_1709_04488_amd import workloads as W

GOLD = read_golden("paper_values.txt")


def _params(orc, **kw):
    return orc.Params(**{**W.default_setup(), **kw})


# --- independent lattice sum (mpmath, 30 digits) -------------------------------

def _m4(q):
    q = mp.mpf(q)
    if q < 1:
        return 1 - mp.mpf(3) / 2 * q ** 2 + mp.mpf(3) / 4 * q ** 3
    if q < 2:
        return (2 - q) ** 3 / 4
    return mp.mpf(0)


def _m4d(q):
    q = mp.mpf(q)
    if q < 1:
        return -3 * q + mp.mpf(9) / 4 * q ** 2
    if q < 2:
        return -mp.mpf(3) / 4 * (2 - q) ** 2
    return mp.mpf(0)


def _lattice_shells(kmax):
    r = []
    for a in range(-kmax, kmax + 1):
        for b in range(-kmax, kmax + 1):
            for c in range(-kmax, kmax + 1):
                r.append(mp.sqrt(a * a + b * b + c * c))
    return r


@pytest.fixture(scope="module")
def lattice_solution():
    """s = h/Delta solving sigma sum_k f(|k|/s) = eta^3 on the infinite cubic
    lattice (that is h^3 rho = eta^3 m with m = rho0 Delta^3), by mpmath."""
    mp.mp.dps = 30
    eta = mp.mpf("1.2")
    dist = _lattice_shells(3)
    g = lambda s: sum(_m4(r / s) for r in dist) / mp.pi - eta ** 3
    s = mp.findroot(g, (mp.mpf("1.1"), mp.mpf("1.3")), solver="bisect", tol=mp.mpf(10) ** -25)
    fsum = sum(_m4(r / s) for r in dist)
    qfp = sum((r / s) * _m4d(r / s) for r in dist)
    omega = -qfp / (3 * fsum)
    nngb = sum(1 for r in dist if 0 < r < 2 * s)
    return float(s), float((eta / s) ** 3), float(omega), nngb


def test_lattice_matches_independent_lattice_sum(orc, lattice_solution):
    s, rho_rel, omega, nngb = lattice_solution
    n = 12
    w = W.lattice(n)
    a = w.arrays
    d = orc.density(_params(orc), a["x"], a["y"], a["z"], a["m"], a["h"])
    assert np.max(np.abs(d["h"] * n / s - 1.0)) < 1e-12
    assert np.max(np.abs(d["rho"] / rho_rel - 1.0)) < 1e-12
    assert np.max(np.abs(d["omega"] / omega - 1.0)) < 1e-12
    assert np.all(d["nngb"] == nngb)


def test_lattice_density_offset_below_paper_bound(orc):
    # section 6.1: the SPH density sum of a uniform set is offset by < 1 %
    w = W.lattice(10)
    a = w.arrays
    for eta in (1.2, 1.5):
        d = orc.density(_params(orc, eta=eta), a["x"], a["y"], a["z"], a["m"], a["h"])
        off = d["rho"] - 1.0
        assert np.ptp(off) < 1e-13
        assert 0.0 < abs(off[0]) < GOLD["density_offset_bound"]


def test_default_eta_gives_about_58_neighbours(orc):
    # eta = 1.2 (section 2.1.1): (4 pi / 3)(2 eta)^3 = 57.9 neighbours in a
    # uniform medium; a perfect lattice gives 56 + self
    eta = GOLD["eta_sph_default"]
    assert abs(4.0 / 3.0 * np.pi * (2 * eta) ** 3 - 57.9) < 0.05
    w = W.config0()
    a = w.arrays
    d = orc.density(_params(orc), a["x"], a["y"], a["z"], a["m"], a["h"])
    assert 50 < d["nngb"].mean() < 70


def test_h_rho_relation_at_convergence(orc):
    w = W.config0()
    a = w.arrays
    p = _params(orc)
    d = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])
    rel = d["h"] ** 3 * d["rho"] / (p.eta ** 3 * a["m"]) - 1.0
    assert np.max(np.abs(rel)) < 1e-13


def test_root_independent_of_guess(orc):
    w = W.jittered_lattice(8, seed=5)
    a = w.arrays
    p = _params(orc)
    ref = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])["h"]
    for fac in (0.2, 0.9, 3.5):
        h = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"] * fac)["h"]
        assert np.max(np.abs(h / ref - 1.0)) < 4e-15


def test_octahedron_centre_closed_form(orc):
    # centre + 6 particles at distance r on the axes, isolated.  For the centre
    # sigma m (f(0) + 6 f(r/h)) = eta^3 m, i.e. f(q) = (pi eta^3 - 1)/6 with
    # q = r/h < 1: 1 - 1.5 q^2 + 0.75 q^3 = target, a cubic solved by numpy.
    eta, r = 1.2, 0.37
    target = (np.pi * eta ** 3 - 1.0) / 6.0
    roots = np.roots([0.75, -1.5, 0.0, 1.0 - target])
    q = [z.real for z in roots if abs(z.imag) < 1e-12 and 0 < z.real < 1][0]
    x = np.array([0.0, r, -r, 0, 0, 0, 0])
    y = np.array([0.0, 0, 0, r, -r, 0, 0])
    z = np.array([0.0, 0, 0, 0, 0, r, -r])
    m = np.full(7, 0.25)
    p = _params(orc, periodic=False)
    d = orc.density(p, x, y, z, m, np.full(7, 0.3))
    assert d["h"][0] == pytest.approx(r / q, rel=1e-13)
    assert d["nngb"][0] == 6


def test_too_few_particles_has_no_root(orc):
    # open set: the root exists only if sigma sum_j m_j > eta^3 m_i, i.e. N >= 6
    # for equal masses (1/pi * 5 < 1.728)
    rng = np.random.default_rng(0)
    x, y, z = rng.uniform(0, 1, (3, 5))
    p = _params(orc, periodic=False)
    with pytest.raises(orc.OracleError) as e:
        orc.density(p, x, y, z, np.full(5, 0.2), np.full(5, 0.3))
    assert e.value.code == orc.ORC_ENOROOT


def test_periodic_box_too_small_is_reported(orc):
    w = W.lattice(2)
    a = w.arrays
    with pytest.raises(orc.OracleError) as e:
        orc.density(_params(orc), a["x"], a["y"], a["z"], a["m"], a["h"])
    assert e.value.code == orc.ORC_EBOX


def test_density_and_lists_match_library_neighbour_search(orc):
    # scipy's periodic KD-tree finds the pairs; the pinned kernel weights them
    w = W.jittered_lattice(10, seed=11)
    a = w.arrays
    p = _params(orc)
    d = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])
    pts = np.stack([a["x"], a["y"], a["z"]], 1)
    tree = cKDTree(pts, boxsize=1.0)
    off, idx = orc.neighbours(p, a["x"], a["y"], a["z"], d["h"], mode=0)
    for i in range(0, w.n, 7):
        js = sorted(j for j in tree.query_ball_point(pts[i], 2.0 * d["h"][i]) if j != i)
        assert js == idx[off[i]:off[i + 1]].tolist()
        dd = pts[js + [i]] - pts[i]
        dd -= np.round(dd)
        r = np.sqrt((dd ** 2).sum(1))
        rho = sum(a["m"][j] * orc.kernel_W(rr, d["h"][i]) for j, rr in zip(js + [i], r))
        assert rho == pytest.approx(d["rho"][i], rel=1e-13)


def test_force_lists_are_union_of_both_gather_radii(orc):
    w = W.jittered_lattice(8, seed=3)
    a = w.arrays
    p = _params(orc)
    rng = np.random.default_rng(1)
    h = a["h"] * rng.uniform(0.7, 1.4, w.n)
    o0, i0 = orc.neighbours(p, a["x"], a["y"], a["z"], h, mode=0)
    o1, i1 = orc.neighbours(p, a["x"], a["y"], a["z"], h, mode=1)
    sets0 = [set(i0[o0[i]:o0[i + 1]].tolist()) for i in range(w.n)]
    for i in range(w.n):
        expect = sets0[i] | {j for j in range(w.n) if i in sets0[j]}
        assert expect == set(i1[o1[i]:o1[i + 1]].tolist())


@pytest.mark.parametrize("eps", [1e-6])
def test_drho_dh_and_omega_by_finite_differences(orc, eps):
    w = W.jittered_lattice(6, seed=2)
    a = w.arrays
    p = _params(orc)
    d = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])
    sel = np.arange(0, w.n, 5)
    h = d["h"][sel]
    up = orc.rho_at(p, a["x"], a["y"], a["z"], a["m"], h * (1 + eps), sel=sel)["rho"]
    dn = orc.rho_at(p, a["x"], a["y"], a["z"], a["m"], h * (1 - eps), sel=sel)["rho"]
    fd = (up - dn) / (2 * eps * h)
    assert np.max(np.abs(fd - d["drhodh"][sel]) / np.abs(d["drhodh"][sel])) < 1e-6
    # EQN:OMEGA with dh/drho = -h/(3 rho) from EQN:HRHO
    om = 1.0 - (-h / (3.0 * d["rho"][sel])) * fd
    assert np.max(np.abs(om - d["omega"][sel])) < 1e-7
