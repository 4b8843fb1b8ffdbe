"""Pins of the oracle's hierarchical block time-steps (section 2.1.4) and
time-step limiter (section 2.1.5).

* With every particle on level 0 (time-steps within a factor 2 of each
  other, so dt_max = min_i dt_i) every level-0 step is exactly one global
  kick-drift-kick step: the block integrator reproduces the global one bit
  for bit over several steps.
* Elapsed time after a level-0 step is its dt_max = min_i dt_i 2^k, k the
  largest integer keeping it <= max_i dt_i (of the initial state).
* A few hot particles (short steps) sit on the deepest level, the deepest
  level sets the number of sub-steps, and the particle updates are far
  fewer than a global integration with the same number of steps makes.
* The limiter bounds the level spread between force neighbours (to one
  more than its setting, the lag of one sub-step), which without it grows
  to 3 or more levels here, at the price of more particle updates.
* Energy changes by less than 1e-4 over two level-0 steps (a dissipative
  but smooth set; the global integrator's change is of the same order).
"""
import numpy as np
import pytest

from paper_1709_04488_amd import workloads as W


def _run_block(orc, w, u=None, nfull=1, lim=2, lmax=20):
    a = w.arrays
    p = orc.Params(**w.setup)
    return orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"],
                         a["u"] if u is None else u, a["h"], nfull, lmax=lmax, lim=lim)


def test_single_level_equals_global_kdk(orc):
    w = W.jittered_lattice(7, seed=11, sigma_v=0.01)
    a = w.arrays
    p = orc.Params(**w.setup)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    assert np.min(ev["dt"]) > 0.5 * np.max(ev["dt"])   # every particle on level 0
    st, e, nsub, lev, t = _run_block(orc, w, nfull=3)
    assert nsub == 3 and np.all(lev == 0)
    g, eg, dts = orc.kdk(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"],
                         a["h"], 3, 0.0)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h"):
        assert np.array_equal(st[k], g[k]), k
    assert np.array_equal(e, eg)
    assert t == pytest.approx(np.sum(dts), rel=1e-15)


def test_level0_step_length(orc):
    w = W.jittered_lattice(8, seed=3)
    a = w.arrays
    u = _hot(w)
    p = orc.Params(**w.setup)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], u, a["h"])
    lo, hi = np.min(ev["dt"]), np.max(ev["dt"])
    k = int(np.floor(np.log2(hi / lo)))
    expect = lo * 2.0 ** k
    assert expect <= hi < 2.0 * expect
    _, _, _, _, t = _run_block(orc, w, u=u, nfull=1)
    assert t == expect


def _hot(w, factor=40.0, count=4):
    u = w.arrays["u"].copy()
    u[:count] *= factor
    return u


def test_hot_particles_go_deep_and_save_steps(orc):
    w = W.jittered_lattice(8, seed=3)
    a = w.arrays
    u = _hot(w)
    p = orc.Params(**w.setup)
    ev = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], u, a["h"])
    st, e, nsub, lev, t = _run_block(orc, w, u=u, nfull=2)
    assert t > np.max(ev["dt"])                    # two level-0 steps of more than max dt / 2
    assert np.all(lev[:4] == lev.max()) and lev.max() >= 2 and np.sum(lev == 0) > 100
    assert nsub == 2 * 2 ** int(lev.max())
    assert st["updates"] < 0.6 * nsub * w.n
    assert abs(e[-1] / e[0] - 1.0) < 1e-4


def test_limiter_bounds_the_level_spread_of_neighbours(orc):
    """With lim = 1, force neighbours end at most lim + 1 levels apart (the
    limiter acts on the levels of the previous sub-step, so the final
    positions can show one more); without it (lim = 99) the hot particles
    sit 3 or more levels below some neighbours, and the limiter costs
    particle updates."""
    w = W.jittered_lattice(9, seed=5)
    a = w.arrays
    u = _hot(w, factor=1000.0, count=3)
    p = orc.Params(**w.setup)
    spread = {}
    updates = {}
    for lim in (1, 99):
        st, _, _, lev, _ = _run_block(orc, w, u=u, nfull=2, lim=lim)
        off, idx = orc.neighbours(p, st["x"], st["y"], st["z"], st["h"], 1)
        i = np.repeat(np.arange(w.n), np.diff(off))
        spread[lim] = int(np.abs(lev[i] - lev[idx]).max())
        updates[lim] = st["updates"]
    assert spread[1] <= 2
    assert spread[99] >= 3
    assert updates[1] > updates[99]
