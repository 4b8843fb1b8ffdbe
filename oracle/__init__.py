"""Brute-force FP64 CPU oracle for the grad-h SPH hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  The arithmetic lives in
``sph_oracle.c`` (plain C, FP64, no FMA contraction, O(N^2) sums over every
particle in index order); this module builds it with gcc and marshals numpy
arrays in and out.

Functions and the passages they follow (GANDALF paper, arXiv:1709.04488):

* ``kernel_f/df/W/dWdr/dWdh`` -- M4 cubic spline, R = 2 (section 2);
  ``quintic_f/df`` -- the quintic spline, R = 3 (section 2), chosen for every
  sum by ``Params.kernel``.
* ``density``    -- eqs. EQN:SPHRHO, EQN:HRHO, EQN:OMEGA (section 2.1.1).
* ``eos``        -- ideal gas P = (gamma-1) rho u (below EQN:GRADHMOMEQN).
* ``forces``     -- eqs. EQN:GRADHMOMEQN, EQN:GRADHENEQN, EQN:MON97ARTVISC,
  EQN:MON97ENERGYDISS (artificial viscosity, and artificial conductivity
  when alpha_ac > 0), signal speed and EQN:SPH_DT.
* ``neighbours`` -- the neighbour sets those sums run over.
* ``kdk``        -- eqs. EQN:LFKDK1/EQN:LFKDK2 with the section 5.1 loop order.
* ``kdk_block``  -- the same with hierarchical block time-steps (section
  2.1.4) and the predictive/reactive limiter (section 2.1.5).
* ``mfv``        -- meshless finite-volume geometry (section 2.2): number
  density and h (EQN:MFV_NDENS, EQN:MFV_HN), gradient matrix E
  (EQN:MFVEMATRIX), B = E^-1, least-squares gradients (EQN:MFVGRADIENT,
  EQN:MFVPSI) with the SPH fallback above condition number 100.
* ``mm97_rate``, ``cd10_update`` -- the artificial-viscosity switches section
  2.1.1 names (Morris & Monaghan 1997; Cullen & Dehnen 2010), in their
  published forms; ``forces`` takes per-particle alpha and returns the
  velocity divergence and curl they use.
* ``sampled_evaluation`` -- the same quantities for a few particles of a
  large set, each computed one by one from its own neighbourhood.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ENOROOT, ORC_EBOX, ORC_ECAP = 0, -1, -2, -4, -5, -8


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile sph_oracle.c into liboracle.so (gcc -O2 -fopenmp -ffp-contract=off)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        for name in ("orc_f", "orc_df", "orc_quintic_f", "orc_quintic_df"):
            getattr(lib, name).restype = d
            getattr(lib, name).argtypes = [d]
        for name in ("orc_W", "orc_dWdr", "orc_dWdh"):
            getattr(lib, name).restype = d
            getattr(lib, name).argtypes = [d, d]
        lib.orc_density.restype = ctypes.c_int
        lib.orc_density.argtypes = [vp, i64] + [vp] * 5 + [i64, vp] + [vp] * 5
        lib.orc_rho_at.restype = ctypes.c_int
        lib.orc_rho_at.argtypes = [vp, i64] + [vp] * 4 + [i64, vp, vp, vp, vp, vp]
        lib.orc_eos.restype = None
        lib.orc_eos.argtypes = [i64, d, vp, vp, vp, vp]
        lib.orc_forces.restype = ctypes.c_int
        lib.orc_forces.argtypes = [vp, i64] + [vp] * 11 + [i64, vp] + [vp] * 12
        lib.orc_neighbours.restype = ctypes.c_int
        lib.orc_neighbours.argtypes = [vp, i64, vp, vp, vp, vp, i32, i64, vp, vp, vp, i64]
        lib.orc_kdk.restype = ctypes.c_int
        lib.orc_kdk.argtypes = [vp, i64] + [vp] * 9 + [i32, d, vp, vp, vp]
        lib.orc_mm97_rate.restype = None
        lib.orc_mm97_rate.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        lib.orc_cd10_update.restype = None
        lib.orc_cd10_update.argtypes = [vp, i64, d] + [vp] * 7
        lib.orc_mfv_gradients.restype = ctypes.c_int
        lib.orc_mfv_gradients.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, i64, vp, vp, vp, vp]
        lib.orc_kdk_block.restype = ctypes.c_int
        lib.orc_kdk_block.argtypes = [vp, i64] + [vp] * 9 + [i32, i32, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


class _CParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("ccfl", ctypes.c_double), ("periodic", ctypes.c_int32),
                ("ac_signal", ctypes.c_int32), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("alpha_ac", ctypes.c_double),
                ("av_switch", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("av_ell", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("pad2_", ctypes.c_int32)]

AV_NONE, AV_MM97, AV_CD10 = 0, 1, 2
KERNEL_M4, KERNEL_QUINTIC = 0, 1
# published decay constants: MM97 tau = h/(0.1 c); CD10 tau = h/(2 0.05 v_sig)
AV_ELL_DEFAULT = {AV_MM97: 0.1, AV_CD10: 0.05}


@dataclass
class Params:
    """Method parameters.  Defaults: eta = 1.2 (section 2.1.1), gamma = 5/3,
    alpha_AV = 1, beta_AV = 2 alpha_AV (section 2.1.1), C_CFL = 0.2
    (section 2.1.4), no artificial conductivity (alpha_AC = 0; eq.
    EQN:MON97ENERGYDISS).  ac_signal picks the conductivity signal speed:
    0 = Wadsley 2008 |v_ij . rhat_ij| (the paper's default), 1 = Price 2008
    sqrt(|P_i - P_j| / rhobar_ij)."""
    eta: float = 1.2
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    ccfl: float = 0.2
    periodic: bool = True
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    alpha_ac: float = 0.0
    ac_signal: int = 0
    av_switch: int = 0          # AV_NONE, AV_MM97 or AV_CD10
    alpha_min: float = 0.1
    alpha_max: float = 1.0
    av_ell: float = 0.0         # 0: the switch's published value
    kernel: int = 0             # KERNEL_M4 (R = 2) or KERNEL_QUINTIC (R = 3)

    def support(self) -> float:
        """The kernel's support radius in units of h (section 2)."""
        return 3.0 if self.kernel == KERNEL_QUINTIC else 2.0

    def c(self) -> _CParams:
        p = _CParams()
        p.eta, p.gamma, p.alpha, p.beta, p.ccfl = self.eta, self.gamma, self.alpha, self.beta, self.ccfl
        p.periodic = 1 if self.periodic else 0
        p.ac_signal = int(self.ac_signal)
        p.alpha_ac = float(self.alpha_ac)
        p.av_switch = int(self.av_switch)
        p.alpha_min, p.alpha_max = float(self.alpha_min), float(self.alpha_max)
        p.av_ell = float(self.av_ell) if self.av_ell > 0.0 else AV_ELL_DEFAULT.get(self.av_switch, 0.0)
        p.kernel = int(self.kernel)
        for k in range(3):
            p.lo[k] = float(self.lo[k])
            p.hi[k] = float(self.hi[k])
        return p


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --- kernel -----------------------------------------------------------------

def kernel_f(q: float) -> float:
    return _load().orc_f(float(q))


def kernel_df(q: float) -> float:
    return _load().orc_df(float(q))


def kernel_W(r: float, h: float) -> float:
    return _load().orc_W(float(r), float(h))


def kernel_dWdr(r: float, h: float) -> float:
    return _load().orc_dWdr(float(r), float(h))


def kernel_dWdh(r: float, h: float) -> float:
    return _load().orc_dWdh(float(r), float(h))


def quintic_f(q: float) -> float:
    """Quintic spline shape (Morris 1996), support R = 3 (section 2)."""
    return _load().orc_quintic_f(float(q))


def quintic_df(q: float) -> float:
    return _load().orc_quintic_df(float(q))


# --- density, EOS, forces -----------------------------------------------------

def density(params: Params, x, y, z, m, h_guess, sel=None) -> dict:
    """h, rho, drho/dh (= sum m dW/dh), omega, nngb for each selected particle."""
    lib = _load()
    x, y, z, m, hg = (_f64(a) for a in (x, y, z, m, h_guess))
    n = x.size
    sel_a = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    k = n if sel_a is None else sel_a.size
    out = {key: np.empty(k, np.float64) for key in ("h", "rho", "drhodh", "omega")}
    out["nngb"] = np.empty(k, np.int32)
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_density(ctypes.byref(cp), n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(hg),
                         k, _ptr(sel_a), _ptr(out["h"]), _ptr(out["rho"]), _ptr(out["drhodh"]),
                         _ptr(out["omega"]), _ptr(out["nngb"]))
    if rc != ORC_OK:
        raise OracleError(rc, "density")
    return out


def rho_at(params: Params, x, y, z, m, h, sel=None) -> dict:
    """rho, drho/dh and density-neighbour count at the given h (no solve);
    ``h`` is indexed like the selection."""
    lib = _load()
    x, y, z, m = (_f64(a) for a in (x, y, z, m))
    n = x.size
    sel_a = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    k = n if sel_a is None else sel_a.size
    hs = _f64(h)
    assert hs.size == k
    out = {"rho": np.empty(k), "drhodh": np.empty(k), "nngb": np.empty(k, np.int32)}
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_rho_at(ctypes.byref(cp), n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), k, _ptr(sel_a),
                        _ptr(hs), _ptr(out["rho"]), _ptr(out["drhodh"]), _ptr(out["nngb"]))
    if rc != ORC_OK:
        raise OracleError(rc, "rho_at")
    return out


def eos(gamma: float, rho, u):
    lib = _load()
    rho, u = _f64(rho), _f64(u)
    P = np.empty_like(rho)
    c = np.empty_like(rho)
    lib.orc_eos(rho.size, float(gamma), _ptr(rho), _ptr(u), _ptr(P), _ptr(c))
    return P, c


def forces(params: Params, x, y, z, vx, vy, vz, m, u, h, rho, omega, sel=None,
           alpha=None) -> dict:
    """a, du/dt, v_sig, dt_i, per-particle scales, force-neighbour counts,
    velocity divergence and curl; alpha: per-particle viscosity strengths
    (pair value (alpha_i + alpha_j)/2), default alpha_AV everywhere."""
    lib = _load()
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m, u, h, rho, omega)]
    n = arrs[0].size
    sel_a = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    k = n if sel_a is None else sel_a.size
    keys = ("ax", "ay", "az", "dudt", "vsig", "dt", "scale_a", "scale_u")
    out = {key: np.empty(k, np.float64) for key in keys}
    out["nforce"] = np.empty(k, np.int32)
    out["divv"] = np.empty(k, np.float64)
    out["curlv"] = np.empty(k, np.float64)
    al = None if alpha is None else _f64(alpha)
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_forces(ctypes.byref(cp), n, *[_ptr(a) for a in arrs], k, _ptr(sel_a),
                        *[_ptr(out[key]) for key in keys], _ptr(out["nforce"]), _ptr(al),
                        _ptr(out["divv"]), _ptr(out["curlv"]))
    if rc != ORC_OK:
        raise OracleError(rc, "forces")
    return out


def evaluate(params: Params, x, y, z, vx, vy, vz, m, u, h_guess, alpha=None) -> dict:
    """Full evaluation: density (h solve), EOS, forces, for every particle."""
    d = density(params, x, y, z, m, h_guess)
    P, c = eos(params.gamma, d["rho"], u)
    f = forces(params, x, y, z, vx, vy, vz, m, u, d["h"], d["rho"], d["omega"], alpha=alpha)
    out = dict(d)
    out.update(f)
    out["P"], out["cs"] = P, c
    return out


def neighbours(params: Params, x, y, z, h, mode: int, sel=None):
    """CSR neighbour lists (ascending j) -> (offsets[int64, k+1], idx[int32])."""
    lib = _load()
    x, y, z, h = (_f64(a) for a in (x, y, z, h))
    n = x.size
    sel_a = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    k = n if sel_a is None else sel_a.size
    counts = np.empty(k, np.int64)
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_neighbours(ctypes.byref(cp), n, _ptr(x), _ptr(y), _ptr(z), _ptr(h), int(mode),
                            k, _ptr(sel_a), _ptr(counts), None, 0)
    if rc != ORC_OK:
        raise OracleError(rc, "neighbours")
    total = int(counts.sum())
    idx = np.empty(max(total, 1), np.int32)
    rc = lib.orc_neighbours(ctypes.byref(cp), n, _ptr(x), _ptr(y), _ptr(z), _ptr(h), int(mode),
                            k, _ptr(sel_a), _ptr(counts), _ptr(idx), total)
    if rc != ORC_OK:
        raise OracleError(rc, "neighbours")
    off = np.zeros(k + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return off, idx[:total]


def kdk(params: Params, x, y, z, vx, vy, vz, m, u, h_guess, nsteps: int, dt_fixed: float = 0.0,
        alpha=None):
    """Integrate nsteps KDK steps.  Returns (state dict, energy[nsteps+1], dt[nsteps]).
    With an AV switch, alpha holds the initial per-particle strengths and the
    state dict the final ones (key "alpha")."""
    lib = _load()
    st = {k: _f64(a).copy() for k, a in zip(("x", "y", "z", "vx", "vy", "vz", "u", "h"),
                                           (x, y, z, vx, vy, vz, u, h_guess))}
    m = _f64(m)
    n = m.size
    if params.av_switch:
        st["alpha"] = _f64(alpha if alpha is not None else np.full(n, params.alpha_max)).copy()
    energy = np.empty(nsteps + 1, np.float64)
    dts = np.empty(max(nsteps, 1), np.float64)
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_kdk(ctypes.byref(cp), n, _ptr(st["x"]), _ptr(st["y"]), _ptr(st["z"]),
                     _ptr(st["vx"]), _ptr(st["vy"]), _ptr(st["vz"]), _ptr(m), _ptr(st["u"]),
                     _ptr(st["h"]), int(nsteps), float(dt_fixed), _ptr(energy), _ptr(dts),
                     _ptr(st.get("alpha")))
    if rc != ORC_OK:
        raise OracleError(rc, "kdk")
    return st, energy, dts[:nsteps]


def kdk_block(params: Params, x, y, z, vx, vy, vz, m, u, h_guess, nfull: int, lmax: int = 20,
              lim: int = 2, alpha=None):
    """Block time-step KDK over nfull level-0 steps.  Returns (state dict,
    energy[nfull+1] at the full synchronisations, sub-steps, levels, time);
    the state dict also holds "updates", the active particles summed over
    the sub-steps.  With an AV switch, alpha holds the initial per-particle
    strengths (default alpha_max) and the state dict the final ones (key
    "alpha")."""
    lib = _load()
    st = {k: _f64(a).copy() for k, a in zip(("x", "y", "z", "vx", "vy", "vz", "u", "h"),
                                           (x, y, z, vx, vy, vz, u, h_guess))}
    m = _f64(m)
    n = m.size
    if params.av_switch:
        st["alpha"] = _f64(alpha if alpha is not None else np.full(n, params.alpha_max)).copy()
    energy = np.empty(nfull + 1)
    nsub = ctypes.c_int64(0)
    tout = ctypes.c_double(0.0)
    upd = ctypes.c_int64(0)
    lev = np.empty(n, np.int32)
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_kdk_block(ctypes.byref(cp), n, _ptr(st["x"]), _ptr(st["y"]), _ptr(st["z"]),
                           _ptr(st["vx"]), _ptr(st["vy"]), _ptr(st["vz"]), _ptr(m), _ptr(st["u"]),
                           _ptr(st["h"]), int(lmax), int(lim), int(nfull), _ptr(energy),
                           ctypes.byref(nsub), _ptr(lev), ctypes.byref(tout), ctypes.byref(upd),
                           _ptr(st.get("alpha")))
    if rc != ORC_OK:
        raise OracleError(rc, "kdk_block")
    st["updates"] = int(upd.value)
    return st, energy, int(nsub.value), lev, float(tout.value)


def mm97_rate(params: Params, alpha, divv, c, h):
    """d alpha / dt of the Morris & Monaghan 1997 switch."""
    lib = _load()
    arrs = [_f64(a) for a in (alpha, divv, c, h)]
    out = np.empty_like(arrs[0])
    cp = _CParams.from_buffer_copy(params.c())
    lib.orc_mm97_rate(ctypes.byref(cp), arrs[0].size, *[_ptr(a) for a in arrs], _ptr(out))
    return out


def cd10_update(params: Params, dt: float, alpha, divv, divv_prev, curlv, vsig, c, h):
    """alpha after one step of length dt under the Cullen & Dehnen 2010 switch."""
    lib = _load()
    al = _f64(alpha).copy()
    arrs = [_f64(a) for a in (divv, divv_prev, curlv, vsig, c, h)]
    cp = _CParams.from_buffer_copy(params.c())
    lib.orc_cd10_update(ctypes.byref(cp), al.size, float(dt), _ptr(al), *[_ptr(a) for a in arrs])
    return al


def mfv(params: Params, x, y, z, h_guess, fields=(), sel=None) -> dict:
    """Number density n, h, B = E^-1 (xx, xy, xz, yy, yz, zz), condition
    number and the gradients of each field (shape [k, nfields, 3])."""
    lib = _load()
    x, y, z = (_f64(a) for a in (x, y, z))
    n = x.size
    ones = np.ones(n)
    d = density(params, x, y, z, ones, h_guess)            # h^3 n = eta^3
    sel_a = None if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    k = n if sel_a is None else sel_a.size
    fl = [_f64(f) for f in fields]
    fp = (ctypes.c_void_p * max(len(fl), 1))(*[f.ctypes.data for f in fl])
    B = np.empty((k, 6))
    cond = np.empty(k)
    grad = np.empty((k, max(len(fl), 1), 3))
    cp = _CParams.from_buffer_copy(params.c())
    rc = lib.orc_mfv_gradients(ctypes.byref(cp), n, _ptr(x), _ptr(y), _ptr(z), _ptr(d["h"]),
                               _ptr(d["rho"]), len(fl), fp, k, _ptr(sel_a), _ptr(B), _ptr(cond),
                               _ptr(grad))
    if rc != ORC_OK:
        raise OracleError(rc, "mfv")
    pick = slice(None) if sel_a is None else sel_a
    return {"h": d["h"][pick], "ndens": d["rho"][pick], "nngb": d["nngb"][pick], "B": B,
            "cond": cond, "grad": grad[:, :len(fl), :]}


# --- sampled evaluation for sets too large for O(N^2) -------------------------

def _min_image_dist2(params: Params, x, y, z, xi, yi, zi):
    d2 = np.zeros(x.size, np.float64)
    for arr, ci, k in ((x, xi, 0), (y, yi, 1), (z, zi, 2)):
        d = ci - arr
        if params.periodic:
            L = params.hi[k] - params.lo[k]
            d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
        d2 += d * d
    return d2


@dataclass
class SampledResult:
    sample: np.ndarray
    force_sample: np.ndarray = None
    values: dict = field(default_factory=dict)
    n_dens: np.ndarray = None
    n_force: np.ndarray = None
    seconds: float = 0.0
    closure_particles: int = 0


def _local_density(params: Params, x, y, z, m, hg, d2, targets, Rs):
    """Density of ``targets`` computed over the particles within Rs of the
    centre whose squared distances are ``d2``.  The solver only evaluates
    smoothing lengths up to max(guess, 2 root); once the support of every such
    h lies inside the sub-set, every sum it formed equals the sum over all N
    (the kernel vanishes beyond R h), so the result is the full-set result."""
    r_t = np.sqrt(d2[targets])
    Rk = params.support()
    while True:
        sub = np.nonzero(d2 < Rs * Rs)[0]
        dd = density(params, x[sub], y[sub], z[sub], m[sub], hg[sub],
                     sel=np.searchsorted(sub, targets))
        need = r_t + Rk * np.maximum(hg[targets], 2.0 * dd["h"])
        if np.all(need < Rs):
            return dd
        Rs = float(np.max(need)) * 1.5


def sampled_evaluation(params: Params, arrays: dict, sample, force_sample=None,
                       alpha=None) -> SampledResult:
    """Oracle values for a few particles of a large set, one particle at a time.

    Density, h, omega, P, c for every particle of ``sample`` (each h is the
    root of its own h-rho relation over all N particles); forces, du/dt,
    v_sig and dt for ``force_sample`` (default: ``sample``).  With the kernel's
    support radius Rk (2 for M4, 3 for the quintic), forces on i need h, rho,
    omega of every j with r_ij < Rk max(h_i, h_j); those j are found by
    growing a radius R around i until every particle inside R has
    Rk h_j <= R, and by also solving exactly every particle whose input guess
    would reach i with 25 % to spare (1.25 Rk h_guess_j > r_ij).  The guesses
    only choose which particles get an exact root; they never enter a sum.
    This closure assumes that no other particle has a smoothing length larger
    than half its distance to i, which holds for the smooth density fields of
    the synthetic workloads.  alpha: per-particle viscosity strengths (the AV
    switches), indexed like the arrays.
    """
    t0 = time.perf_counter()
    x, y, z = (_f64(arrays[k]) for k in ("x", "y", "z"))
    vx, vy, vz = (_f64(arrays[k]) for k in ("vx", "vy", "vz"))
    m, u, hg = _f64(arrays["m"]), _f64(arrays["u"]), _f64(arrays["h"])
    sample = np.asarray(sample, dtype=np.int64)
    fsample = sample if force_sample is None else np.asarray(force_sample, dtype=np.int64)
    res = SampledResult(sample=sample, force_sample=fsample)
    Rk = params.support()

    d = density(params, x, y, z, m, hg, sel=sample)
    P, c = eos(params.gamma, d["rho"], u[sample])
    res.values.update({"h": d["h"], "rho": d["rho"], "omega": d["omega"], "P": P, "cs": c,
                       "drhodh": d["drhodh"]})
    res.n_dens = d["nngb"].astype(np.int64)
    known = {int(i): (hh, rr, oo) for i, hh, rr, oo in
             zip(sample.tolist(), d["h"].tolist(), d["rho"].tolist(), d["omega"].tolist())}

    keys = ("ax", "ay", "az", "dudt", "vsig", "dt", "scale_a", "scale_u", "divv", "curlv")
    fvals = {k: np.empty(fsample.size) for k in keys}
    nforce = np.empty(fsample.size, np.int64)
    closure = 0
    for k, i in enumerate(fsample.tolist()):
        d2 = _min_image_dist2(params, x, y, z, x[i], y[i], z[i])
        if i not in known:
            di = _local_density(params, x, y, z, m, hg, d2, np.array([i]),
                                4.0 * Rk * float(hg[i]))
            known[i] = (float(di["h"][0]), float(di["rho"][0]), float(di["omega"][0]))
        R = Rk * known[i][0]
        reach = d2 < (1.25 * Rk * hg) ** 2
        for _ in range(64):
            inside = np.nonzero((d2 < R * R) | reach)[0]
            todo = np.array([j for j in inside.tolist() if j not in known], dtype=np.int64)
            if todo.size:
                Rs = float(np.sqrt(np.max(d2[todo]))) + 4.0 * Rk * max(float(np.max(hg[todo])),
                                                                  known[i][0])
                dd = _local_density(params, x, y, z, m, hg, d2, todo, Rs)
                for j, hh, rr, oo in zip(todo.tolist(), dd["h"].tolist(), dd["rho"].tolist(),
                                         dd["omega"].tolist()):
                    known[j] = (hh, rr, oo)
            core = np.nonzero(d2 < R * R)[0]
            hmax = max(known[j][0] for j in core.tolist())
            if Rk * hmax <= R:
                break
            R = Rk * hmax * (1.0 + 1e-7)
        else:
            raise OracleError(ORC_ENOROOT, "sampled closure")
        hs = np.array([known[j][0] for j in inside.tolist()])
        rs = np.array([known[j][1] for j in inside.tolist()])
        os_ = np.array([known[j][2] for j in inside.tolist()])
        ii = int(np.searchsorted(inside, i))
        fo = forces(params, x[inside], y[inside], z[inside], vx[inside], vy[inside], vz[inside],
                    m[inside], u[inside], hs, rs, os_, sel=[ii],
                    alpha=None if alpha is None else np.asarray(alpha)[inside])
        for key in keys:
            fvals[key][k] = fo[key][0]
        nforce[k] = int(fo["nforce"][0])
        closure += int(inside.size)
    res.values.update(fvals)
    res.n_force = nforce
    res.closure_particles = closure
    res.seconds = time.perf_counter() - t0
    return res
