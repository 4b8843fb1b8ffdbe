"""Seeded synthetic particle sets.

This module only draws random numbers and lays particles out; it holds none
of the method's arithmetic (no kernel, no density sum, no force).  Both the
HIP path's callers and the brute-force oracle take their inputs from here.

Every set is returned as host float64 arrays in structure-of-arrays form:
x, y, z, vx, vy, vz, m, u and h (an initial smoothing-length guess drawn from
the density the recipe was built to have; the converged h does not depend on
it, because the h-rho relation has a unique root).

Recipes (code units, equal masses m = 1/N):

* ``jittered_lattice`` -- n^3 sites at (k + 1/2)/n of the periodic unit box,
  each coordinate jittered by U(-0.1, 0.1)/n, u = u0 (1 + 0.1 U(-1, 1)),
  v ~ N(0, sigma_v^2) per component.
* ``blob_in_lattice`` -- the jittered lattice with a fraction of the particles
  (a seeded permutation) redrawn from a Gaussian blob N(0.5, sigma_b^2) per
  axis, wrapped into the box; u lognormal(0, 0.3), v ~ N(0, 0.2^2).
* ``plummer`` -- a Plummer sphere (density and 1D dispersion as in the
  Plummer-sphere test of section 6.7, eq. EQN:PLUMMERRHO) with scale radius a, radius cut,
  isolated boundary, velocities N(0, sigma^2(r)) per component and
  u = sigma^2(r)/(gamma - 1) (the hybrid star-and-gas Plummer set-up, section 6.8).
* ``lattice`` -- a perfect n^3 cubic lattice, at rest (used by invariants).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ETA = 1.2
GAMMA = 5.0 / 3.0


@dataclass
class Workload:
    name: str
    arrays: dict
    setup: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.arrays["x"].size)


def default_setup(periodic: bool = True, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> dict:
    return {"eta": ETA, "gamma": GAMMA, "alpha": 1.0, "beta": 2.0, "ccfl": 0.2,
            "periodic": bool(periodic), "lo": tuple(float(v) for v in lo),
            "hi": tuple(float(v) for v in hi)}


def _h_guess(m: np.ndarray, rho_guess: np.ndarray) -> np.ndarray:
    return ETA * np.cbrt(m / rho_guess)


def _wrap(a: np.ndarray) -> np.ndarray:
    a = np.mod(a, 1.0)
    # np.mod can return exactly 1.0 for tiny negative inputs
    a[a >= 1.0] = 0.0
    return a


def lattice(n_side: int, spacing_jitter: float = 0.0, seed: int = 0) -> Workload:
    """Perfect (or jittered) n^3 lattice in the periodic unit box, at rest, u = 1."""
    rng = np.random.default_rng(seed)
    k = (np.arange(n_side, dtype=np.float64) + 0.5) / n_side
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    pos = [a.ravel().copy() for a in (X, Y, Z)]
    n = pos[0].size
    if spacing_jitter:
        for a in pos:
            a += rng.uniform(-spacing_jitter, spacing_jitter, n) / n_side
            a[:] = _wrap(a)
    m = np.full(n, 1.0 / n)
    arrays = {"x": pos[0], "y": pos[1], "z": pos[2], "vx": np.zeros(n), "vy": np.zeros(n),
              "vz": np.zeros(n), "m": m, "u": np.ones(n), "h": _h_guess(m, np.ones(n))}
    return Workload(f"lattice{n_side}", arrays, default_setup())


def jittered_lattice(n_side: int, seed: int, u0: float = 1.0, sigma_v: float = 0.1) -> Workload:
    rng = np.random.default_rng(seed)
    k = (np.arange(n_side, dtype=np.float64) + 0.5) / n_side
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    n = n_side ** 3
    pos = []
    for a in (X, Y, Z):
        a = a.ravel() + rng.uniform(-0.1, 0.1, n) / n_side
        pos.append(_wrap(a))
    u = u0 * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, n))
    v = rng.normal(0.0, sigma_v, (3, n))
    m = np.full(n, 1.0 / n)
    arrays = {"x": pos[0], "y": pos[1], "z": pos[2], "vx": v[0].copy(), "vy": v[1].copy(),
              "vz": v[2].copy(), "m": m, "u": u, "h": _h_guess(m, np.ones(n))}
    return Workload(f"jittered_lattice{n_side}", arrays, default_setup())


def blob_in_lattice(n_side: int, seed: int, blob_frac: float = 0.3,
                    sigma_b: float = 0.05) -> Workload:
    rng = np.random.default_rng(seed)
    k = (np.arange(n_side, dtype=np.float64) + 0.5) / n_side
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    n = n_side ** 3
    pos = []
    for a in (X, Y, Z):
        a = a.ravel() + rng.uniform(-0.1, 0.1, n) / n_side
        pos.append(_wrap(a))
    nb = int(round(blob_frac * n))
    idx = rng.permutation(n)[:nb]
    for a in pos:
        a[idx] = _wrap(rng.normal(0.5, sigma_b, nb))
    u = np.exp(rng.normal(0.0, 0.3, n))
    v = rng.normal(0.0, 0.2, (3, n))
    m = np.full(n, 1.0 / n)
    # density the recipe was built to have: uniform background + Gaussian blob
    r2 = (pos[0] - 0.5) ** 2 + (pos[1] - 0.5) ** 2 + (pos[2] - 0.5) ** 2
    rho = (1.0 - blob_frac) + blob_frac * (2 * np.pi * sigma_b ** 2) ** -1.5 * np.exp(
        -0.5 * r2 / sigma_b ** 2)
    arrays = {"x": pos[0], "y": pos[1], "z": pos[2], "vx": v[0].copy(), "vy": v[1].copy(),
              "vz": v[2].copy(), "m": m, "u": u, "h": _h_guess(m, rho)}
    return Workload(f"blob_in_lattice{n_side}", arrays, default_setup())


def plummer(n: int, seed: int, a: float = 0.05, r_cut: float = 1.0) -> Workload:
    """Plummer sphere, G = M = 1, isolated boundary."""
    rng = np.random.default_rng(seed)
    r = np.empty(n)
    filled = 0
    while filled < n:
        X = rng.uniform(0.0, 1.0, n)
        X = X[X > 0.0]
        rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr < r_cut]
        take = min(rr.size, n - filled)
        r[filled:filled + take] = rr[:take]
        filled += take
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    x, y, z = r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth
    sig2 = (1.0 / (6.0 * a)) / np.sqrt(1.0 + (r / a) ** 2)
    v = rng.normal(0.0, 1.0, (3, n)) * np.sqrt(sig2)
    u = sig2 / (GAMMA - 1.0)
    m = np.full(n, 1.0 / n)
    rho = 3.0 / (4.0 * np.pi * a ** 3) * (1.0 + (r / a) ** 2) ** -2.5
    arrays = {"x": x, "y": y, "z": z, "vx": v[0].copy(), "vy": v[1].copy(), "vz": v[2].copy(),
              "m": m, "u": u, "h": _h_guess(m, rho)}
    return Workload(f"plummer{n}", arrays, default_setup(periodic=False))


# --- the five named workloads -------------------------------------------------

def config0() -> Workload:
    """N = 4096: 16^3 jittered lattice, periodic unit box (seed 0)."""
    w = jittered_lattice(16, seed=0)
    w.name = "sph3d_lattice16_fp64"
    return w


def config1(n_side: int = 128) -> Workload:
    """N = 2,097,152: jittered 128^3 lattice + 30 % Gaussian blob (seed 1)."""
    w = blob_in_lattice(n_side, seed=1)
    w.name = f"sph3d_blob_in_lattice{n_side}"
    return w


def config2(n: int = 4_194_304) -> Workload:
    """N = 4,194,304 Plummer sphere, a = 0.05, cut 1.0, isolated (seed 2)."""
    w = plummer(n, seed=2)
    w.name = f"sph3d_plummer{n}"
    return w


def _snap_cube(nv: float) -> int:
    return max(2, int(round(nv ** (1.0 / 3.0))))


def request_sizes(count: int, n_lo: float, n_hi: float, seed: int) -> list:
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))
    return [_snap_cube(v) for v in ns]


def config3_requests(count: int = 512, seed: int = 3):
    """Serving mix: lattice boxes with N log-uniform in [1e3, 2e5] snapped to
    n^3, FP64 or FP32-pair with probability 1/2 each."""
    sides = request_sizes(count, 1e3, 2e5, seed)
    rng = np.random.default_rng(seed + 1)
    prec = rng.integers(0, 2, count)
    return [(s, int(p), 1000 * 3 + rid) for rid, (s, p) in enumerate(zip(sides, prec))]


def config4_requests(count: int = 64, seed: int = 4):
    """Served integration mix: blob-in-lattice boxes, N log-uniform in
    [1e4, 1e6] snapped to n^3."""
    sides = request_sizes(count, 1e4, 1e6, seed)
    return [(s, 1000 * 4 + rid) for rid, s in enumerate(sides)]
