"""Pins of the oracle's viscosity switches under hierarchical block
time-steps (section 2.1.4; the switches section 2.1.1 names).

* Every particle on level 0: the block integrator with MM97 or CD10
  reproduces the global kick-drift-kick integrator with the same switch bit
  for bit (positions, velocities, u and alpha).
* A lattice at rest with a hot slab (u 16 times higher, so c 4 times
  higher and the slab two levels deeper than the cold gas).  Far from the
  slab's faces the gas stays at rest (div v ~ 0 and c/h constant), so:
  - MM97: d alpha/dt = -k (alpha - alpha_min), k = ell c / h, integrated by
    kick-drift-kick over steps of length d (opening kick, predictor to the
    end of the step, rate from the predicted alpha, closing kick) gives
    exactly (alpha - alpha_min) -> (alpha - alpha_min)(1 - k d + (k d)^2 / 2)
    per step, with d the particle's own step: level-2 particles take four
    steps of dt_max / 4, level-0 particles one of dt_max.
  - CD10: with no compression the local target is alpha_min and alpha
    relaxes towards it by exp(-2 ell v_sig d / h) per step (v_sig = 2 c),
    so after the time t of a level-0 step (alpha - alpha_min) falls by
    exp(-4 ell c t / h) on every level.
  Using the level-0 step for a level-2 particle (or the wrong predictor
  interval) misses these by a relative 1e-2 or more.
"""
import numpy as np
import pytest


def _lattice_with_hot_slab(nx=32, ny=8):
    """nx x ny x ny lattice, spacing 1/ny, periodic box [0, nx/ny) x [0, 1)^2,
    at rest; u = 16 for x < nx / (2 ny), else 1."""
    s = 1.0 / ny
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(ny), indexing="ij")
    x = (ix.ravel() + 0.5) * s
    y = (iy.ravel() + 0.5) * s
    z = (iz.ravel() + 0.5) * s
    n = x.size
    Lx = nx * s
    m = np.full(n, Lx / n)          # mean density 1
    u = np.where(x < 0.5 * Lx, 16.0, 1.0)
    h = np.full(n, 1.2 * s)
    zero = np.zeros(n)
    arrays = {"x": x, "y": y, "z": z, "vx": zero.copy(), "vy": zero.copy(), "vz": zero.copy(),
              "m": m, "u": u, "h": h}
    setup = {"eta": 1.2, "gamma": 5.0 / 3.0, "alpha": 1.0, "beta": 2.0, "ccfl": 0.2,
             "periodic": True, "lo": (0.0, 0.0, 0.0), "hi": (Lx, 1.0, 1.0)}
    return arrays, setup


@pytest.mark.parametrize("sw", [1, 2])
def test_single_level_block_switch_equals_global(orc, sw):
    from paper_1709_04488_amd import workloads as W
    w = W.jittered_lattice(7, seed=11, sigma_v=0.01)
    a = w.arrays
    p = orc.Params(**w.setup, av_switch=sw)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    assert np.min(ev["dt"]) > 0.5 * np.max(ev["dt"])   # every particle on level 0
    al0 = np.linspace(0.2, 0.9, w.n)
    st, e, nsub, lev, t = orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                                        a["m"], a["u"], a["h"], 3, alpha=al0)
    assert nsub == 3 and np.all(lev == 0)
    g, eg, dts = orc.kdk(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"],
                         a["h"], 3, 0.0, alpha=al0)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "alpha"):
        assert np.array_equal(st[k], g[k]), k
    assert not np.array_equal(st["alpha"], al0)


def _slab_run(orc, sw):
    a, setup = _lattice_with_hot_slab()
    p = orc.Params(**setup, av_switch=sw)
    al0 = np.full(a["x"].size, p.alpha_max)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    st, e, nsub, lev, t = orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                                        a["m"], a["u"], a["h"], 1, alpha=al0)
    return a, p, ev, st, nsub, lev, t


def _quiet(a, Lx=4.0):
    x = a["x"]
    return np.abs(x - 0.25 * Lx) < 0.07, np.abs(x - 0.75 * Lx) < 0.07   # hot, cold slab middles


@pytest.mark.parametrize("sw", [1, 2])
def test_switch_decay_on_two_levels(orc, sw):
    a, p, ev, st, nsub, lev, t = _slab_run(orc, sw)
    hot, cold = _quiet(a)
    assert hot.sum() == 128 and cold.sum() == 128
    # the faces (c_hot + c_cold, then approach) sit deeper still
    assert np.all(lev[hot] == 2) and np.all(lev[cold] == 0) and nsub >= 4
    dtmax = t
    ell = orc.AV_ELL_DEFAULT[sw]
    c = np.sqrt(p.gamma * (p.gamma - 1.0) * a["u"])
    h = ev["h"]
    a0 = p.alpha_max - p.alpha_min
    got = st["alpha"] - p.alpha_min
    for sel, steps in ((hot, 4), (cold, 1)):
        d = dtmax / steps
        if sw == 1:
            kd = ell * c[sel] / h[sel] * d
            want = a0 * (1.0 - kd + 0.5 * kd * kd) ** steps
        else:
            want = a0 * np.exp(-4.0 * ell * c[sel] * dtmax / h[sel])
        # measured: 2e-16 on the cold level; 2e-7 (MM97) and 8e-8 (CD10) on
        # the hot level, where the faces' motion reaches the middle within its
        # four sub-steps (h there varies by 1e-11); a level-0 step taken by a
        # level-2 particle is off by ~6e-4
        assert np.max(np.abs(got[sel] / want - 1.0)) < 1e-5, (sw, steps)
    # the decay is real (several per cent on the hot level)
    assert np.max(got[hot]) < 0.99 * a0
