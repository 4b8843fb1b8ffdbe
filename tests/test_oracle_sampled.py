"""The sampled oracle (used at sizes where O(N^2) is out of reach) must give
bit-for-bit the full brute-force values on sets small enough for both."""
import numpy as np
import pytest

from paper_1709_04488_amd import workloads as W


@pytest.mark.parametrize("ac", [{}, {"alpha_ac": 1.0, "ac_signal": 1}])
def test_sampled_equals_full_periodic(orc, ac):
    w = W.blob_in_lattice(12, seed=4)
    a = w.arrays
    p = orc.Params(**{**w.setup, **ac})
    full = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    sample = np.random.default_rng(0).choice(w.n, 12, replace=False)
    res = orc.sampled_evaluation(p, a, sample)
    for k in ("h", "rho", "omega", "P", "cs", "ax", "ay", "az", "dudt", "vsig", "dt"):
        np.testing.assert_array_equal(res.values[k], full[k][sample])
    np.testing.assert_array_equal(res.n_dens, full["nngb"][sample])
    np.testing.assert_array_equal(res.n_force, full["nforce"][sample])


def test_sampled_equals_full_open(orc):
    w = W.plummer(1500, seed=6)
    a = w.arrays
    p = orc.Params(**w.setup)
    full = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    sample = np.random.default_rng(1).choice(w.n, 10, replace=False)
    res = orc.sampled_evaluation(p, a, sample)
    for k in ("h", "rho", "ax", "ay", "az", "dudt", "vsig"):
        np.testing.assert_array_equal(res.values[k], full[k][sample])
