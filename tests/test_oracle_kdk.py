"""Pins of the oracle's kick-drift-kick leapfrog (eqs. EQN:LFKDK1,
EQN:LFKDK2): exact free streaming, the position update of EQN:LFKDK1 for the
first step, second-order convergence in dt and energy conservation without
dissipation."""
import numpy as np
import pytest

from paper_1709_04488_amd import workloads as W


def _params(orc, **kw):
    return orc.Params(**{**W.default_setup(), **kw})


def _run(orc, p, a, nsteps, dt, **over):
    b = {**a, **over}
    return orc.kdk(p, b["x"], b["y"], b["z"], b["vx"], b["vy"], b["vz"], b["m"], b["u"], b["h"],
                   nsteps, dt)


def test_uniform_motion_of_a_lattice_is_free_streaming(orc):
    w = W.lattice(6)
    a = w.arrays
    V = (0.31, -0.17, 0.05)
    n = w.n
    st, e, dts = _run(orc, _params(orc), a, 5, 0.01, vx=np.full(n, V[0]), vy=np.full(n, V[1]),
                      vz=np.full(n, V[2]))
    for k, v in zip(("x", "y", "z"), V):
        d = st[k] - a[k] - v * 0.05
        d -= np.round(d)
        assert np.max(np.abs(d)) < 1e-13
    assert np.max(np.abs(st["vx"] - V[0])) < 1e-13
    assert np.ptp(e) < 1e-13


def test_first_step_matches_position_update(orc):
    # r^{n+1} = r^n + v^n dt + a^n dt^2 / 2 (EQN:LFKDK1)
    w = W.jittered_lattice(6, seed=3)
    a = w.arrays
    p = _params(orc)
    out = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    dt = 1e-3
    st, _, _ = _run(orc, p, a, 1, dt)
    for k, vk, ak in (("x", "vx", "ax"), ("y", "vy", "ay"), ("z", "vz", "az")):
        expect = a[k] + a[vk] * dt + 0.5 * out[ak] * dt * dt
        d = st[k] - expect
        d -= np.round(d)
        assert np.max(np.abs(d)) < 1e-14


def test_second_order_convergence(orc):
    w = W.jittered_lattice(5, seed=8)
    a = w.arrays
    p = _params(orc, alpha=0.0, beta=0.0)
    T = 0.02
    finals = []
    for nsteps in (4, 8, 16):
        st, _, _ = _run(orc, p, a, nsteps, T / nsteps)
        finals.append(st)

    def diff(s1, s2):
        d = s1["x"] - s2["x"]
        d -= np.round(d)
        return np.sqrt(np.mean(d ** 2) + np.mean((s1["vx"] - s2["vx"]) ** 2))

    ratio = diff(finals[0], finals[1]) / diff(finals[1], finals[2])
    assert 3.2 < ratio < 4.8


@pytest.mark.parametrize("alpha_ac", [0.0, 1.0])
def test_energy_conserved_without_dissipation(orc, alpha_ac):
    # artificial conductivity only moves thermal energy between particles, so
    # the total energy is still conserved to the integrator's order
    w = W.jittered_lattice(5, seed=12)
    a = w.arrays
    p = _params(orc, alpha=0.0, beta=0.0, alpha_ac=alpha_ac)
    errs = []
    for dt in (2e-3, 1e-3):
        _, e, _ = _run(orc, p, a, int(round(0.02 / dt)), dt)
        errs.append(abs(e[-1] - e[0]) / e[0])
    assert errs[0] < 1e-5
    assert errs[1] < errs[0] / 2.5


def test_courant_step_is_min_over_particles(orc):
    w = W.jittered_lattice(5, seed=1)
    a = w.arrays
    p = _params(orc)
    out = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    _, _, dts = _run(orc, p, a, 1, 0.0)
    assert dts[0] == np.min(out["dt"])
    assert dts[0] == pytest.approx(np.min(p.ccfl * out["h"] / out["vsig"]), rel=1e-15)
