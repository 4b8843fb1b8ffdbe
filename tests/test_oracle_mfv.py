"""Pins of the oracle's meshless finite-volume geometry (section 2.2).

* h and n obey the relation they are defined by, h = eta n^(-1/3) with
  n = sum_j W(r_ij, h) (EQN:MFV_NDENS, EQN:MFV_HN), checked by an
  independent numpy sum of the M4 kernel.
* The least-squares gradient (EQN:MFVGRADIENT with EQN:MFVPSI and
  EQN:MFVEMATRIX) is exact for any linear field on any particle set whose E
  is well conditioned: sum_j (k.d_j) B d_j psi_j = B E k = k.
* On a perfect cubic lattice E is a multiple of the identity (condition
  number 1) by symmetry.
* A planar set has a singular E: the condition number exceeds 100 and the
  gradient falls back to the SPH estimate, which has no component off the
  plane.
* Scaling all positions by s leaves the condition number unchanged and
  divides gradients by s.
"""
import math

import numpy as np
import pytest


def _poisson(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)


def _m4(q):
    q = np.asarray(q)
    return np.where(q < 1, 1 - 1.5 * q ** 2 + 0.75 * q ** 3,
                    np.where(q < 2, 0.25 * (2 - q) ** 3, 0.0))


def test_number_density_relation(orc):
    x, y, z = _poisson(1500, 3)
    p = orc.Params(periodic=True, eta=1.2)
    r = orc.mfv(p, x, y, z, np.full(x.size, 0.08))
    for i in (0, 17, 900):
        d = np.stack([x - x[i], y - y[i], z - z[i]])
        d -= np.round(d)                       # minimum image, unit box
        q = np.sqrt(np.sum(d * d, axis=0)) / r["h"][i]
        n_i = np.sum(_m4(q)) / (math.pi * r["h"][i] ** 3)
        assert n_i == pytest.approx(r["ndens"][i], rel=1e-12)
        assert r["h"][i] == pytest.approx(1.2 * n_i ** (-1.0 / 3.0), rel=1e-12)


def test_gradient_exact_for_linear_fields(orc):
    x, y, z = _poisson(2000, 5)
    p = orc.Params(periodic=False, eta=1.2)
    k1 = np.array([0.3, -1.7, 2.2])
    k2 = np.array([-4.0, 0.5, 0.0])
    f1 = 3.0 + k1[0] * x + k1[1] * y + k1[2] * z
    f2 = -1.0 + k2[0] * x + k2[1] * y + k2[2] * z
    r = orc.mfv(p, x, y, z, np.full(x.size, 0.08), fields=(f1, f2))
    good = r["cond"] <= 100.0
    assert good.mean() > 0.95
    assert np.max(np.abs(r["grad"][good, 0, :] - k1)) < 1e-11
    assert np.max(np.abs(r["grad"][good, 1, :] - k2)) < 1e-11


def test_lattice_matrix_is_isotropic(orc):
    k = (np.arange(10) + 0.5) / 10
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    p = orc.Params(periodic=True, eta=1.2)
    r = orc.mfv(p, x, y, z, np.full(x.size, 0.12))
    B = r["B"]
    assert np.allclose(B[:, 0], B[:, 3], rtol=1e-12) and np.allclose(B[:, 0], B[:, 5], rtol=1e-12)
    assert np.max(np.abs(B[:, [1, 2, 4]])) < 1e-10 * np.max(np.abs(B[:, 0]))
    assert np.allclose(r["cond"], 1.0, rtol=1e-12)


def test_planar_set_falls_back_to_sph_gradient(orc):
    k = np.arange(12, dtype=np.float64)
    X, Y = np.meshgrid(k, k, indexing="ij")
    x, y = X.ravel(), Y.ravel()
    z = np.zeros_like(x)
    p = orc.Params(periodic=False, eta=2.0)
    f = 2.0 * x - 3.0 * y
    r = orc.mfv(p, x, y, z, np.full(x.size, 1.5), fields=(f,))
    assert np.all(r["cond"] > 100.0)
    assert np.all(r["grad"][:, 0, 2] == 0.0)
    inner = (x > 3) & (x < 8) & (y > 3) & (y < 8)
    # the SPH estimate points along the true gradient in the plane's interior
    g = r["grad"][inner, 0, :2]
    cosang = (g @ np.array([2.0, -3.0])) / (np.linalg.norm(g, axis=1) * math.sqrt(13.0))
    assert np.all(cosang > 0.999)


def test_scaling(orc):
    x, y, z = _poisson(1200, 9)
    p = orc.Params(periodic=False, eta=1.2)
    f = np.sin(3 * x) + y * z
    a = orc.mfv(p, x, y, z, np.full(x.size, 0.08), fields=(f,), sel=np.arange(40))
    s = 2.5
    b = orc.mfv(p, s * x, s * y, s * z, np.full(x.size, 0.08 * s), fields=(f,), sel=np.arange(40))
    assert np.allclose(b["h"], s * a["h"], rtol=1e-12)
    assert np.allclose(b["cond"], a["cond"], rtol=1e-9)
    assert np.allclose(b["grad"], a["grad"] / s, rtol=1e-9, atol=1e-12)
