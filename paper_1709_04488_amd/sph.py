"""ctypes binding of libsph.so (see include/sph.h).

Argument marshalling only: PyTorch supplies device memory (float64 / int32
CUDA tensors) and the HIP stream; every step of the hot path runs in the HIP
kernels of libsph.  There is no fallback: if the library is missing or the
tensors are not on the GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK, SPH_EINVAL, SPH_ENOMEM, SPH_EDEVICE, SPH_ENOTCONVERGED = 0, -1, -2, -3, -4
SPH_ESTENCIL, SPH_ENONFINITE, SPH_EBUDGET, SPH_ECAP, SPH_ESTATE = -5, -6, -7, -8, -9
SPH_ELEVEL = -10
SPH_FP64, SPH_FP32_PAIR = 0, 1
SPH_AC_WADSLEY, SPH_AC_PRICE = 0, 1
SPH_AV_NONE, SPH_AV_MM97, SPH_AV_CD10 = 0, 1, 2
SPH_KERNEL_M4, SPH_KERNEL_QUINTIC = 0, 1

STATUS_NAMES = {0: "SPH_OK", -1: "SPH_EINVAL", -2: "SPH_ENOMEM", -3: "SPH_EDEVICE",
                -4: "SPH_ENOTCONVERGED", -5: "SPH_ESTENCIL", -6: "SPH_ENONFINITE",
                -7: "SPH_EBUDGET", -8: "SPH_ECAP", -9: "SPH_ESTATE", -10: "SPH_ELEVEL"}

EXPORTED = ["sph_default_params", "sph_create", "sph_destroy", "sph_set_stream", "sph_set_params",
            "sph_build_cells", "sph_density", "sph_forces", "sph_evaluate", "sph_upload_state",
            "sph_step",
            "sph_download_state", "sph_state_info", "sph_neighbours", "sph_sync",
            "sph_last_error", "sph_device_bytes", "sph_enable_kernel_timing", "sph_kernel_times",
            "sph_batch_density", "sph_batch_forces", "sph_batch_evaluate", "sph_batch_step",
            "sph_batch_substep",
            "sph_capture_steps",
            "sph_replay_steps", "sph_plan_bytes", "sph_evaluate_noalloc", "sph_noalloc_max_n",
            "sph_mfv_gradients", "sph_substep", "sph_server_create", "sph_server_submit",
            "sph_server_wait", "sph_server_release", "sph_server_slot_bytes",
            "sph_server_plan_bytes", "sph_server_destroy"]


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha_av", ctypes.c_double), ("beta_av", ctypes.c_double),
                ("c_cfl", ctypes.c_double), ("h_rtol", ctypes.c_double),
                ("h_max_iter", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("box_lo", ctypes.c_double * 3), ("box_hi", ctypes.c_double * 3),
                ("precision", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("alpha_ac", ctypes.c_double), ("ac_signal", ctypes.c_int32),
                ("av_switch", ctypes.c_int32), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("av_ell", ctypes.c_double),
                ("block_lmax", ctypes.c_int32), ("block_lim", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("stage_leaves", ctypes.c_int32),
                ("claim_leaves", ctypes.c_int32), ("pad_", ctypes.c_int32)]


SPH_REQUEST_EVALUATE, SPH_REQUEST_INTEGRATE = 0, 1
REQUEST_ERROR_LEN = 160
NIN = 9           # x .. h: a request's inputs, the first FP64 fields


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


class _Particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in (
        "x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "rho", "omega", "pressure", "cs",
        "ax", "ay", "az", "dudt", "vsig", "dt", "nngb", "nforce", "alpha", "divv", "curlv",
        "level")]


class _MfvSet(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("h", ctypes.c_void_p), ("ndens", ctypes.c_void_p),
                ("nngb", ctypes.c_void_p), ("B", ctypes.c_void_p * 6), ("cond", ctypes.c_void_p),
                ("nfields", ctypes.c_int32), ("f", ctypes.c_void_p * 4),
                ("grad", ctypes.c_void_p * 12)]


class _Stats(ctypes.Structure):
    _fields_ = [("time", ctypes.c_double), ("dt_last", ctypes.c_double),
                ("dt_next", ctypes.c_double), ("kinetic", ctypes.c_double),
                ("thermal", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("steps", ctypes.c_int64), ("n_dens_pairs", ctypes.c_int64),
                ("n_force_pairs", ctypes.c_int64), ("dens_pair_evals", ctypes.c_int64),
                ("force_pair_evals", ctypes.c_int64), ("nr_iter_max", ctypes.c_int32),
                ("walk_overflows", ctypes.c_int32), ("dens_leaf_visits", ctypes.c_int64),
                ("dens_walks", ctypes.c_int64), ("nr_iter_total", ctypes.c_int64),
                ("dens_candidate_tests", ctypes.c_int64), ("dens_box_tests", ctypes.c_int64),
                ("force_candidate_tests", ctypes.c_int64), ("force_box_tests", ctypes.c_int64),
                ("density_walk_overflows", ctypes.c_int32), ("force_walk_overflows", ctypes.c_int32),
                ("dens_list_overflows", ctypes.c_int64),
                ("block_full_steps", ctypes.c_int64), ("block_substeps", ctypes.c_int64),
                ("block_active", ctypes.c_int64), ("block_updates", ctypes.c_int64),
                ("block_time", ctypes.c_double), ("block_dt_max", ctypes.c_double),
                ("block_synchronised", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nsteps", ctypes.c_int32), ("params", _Params),
                ("n", ctypes.c_int64), ("in_", ctypes.c_void_p * NIN),
                ("out", ctypes.c_void_p * 19), ("iout", ctypes.c_void_p * 2),
                ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("interactions", ctypes.c_int64), ("info", _Stats),
                ("host_seconds", ctypes.c_double * 4),
                ("error", ctypes.c_char * REQUEST_ERROR_LEN)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> ctypes.CDLL:
    """Load libsph.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1709_04488_amd.build_lib.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER(_Params)
    PS = ctypes.POINTER(_Particles)
    sig = {
        "sph_default_params": (None, [P]),
        "sph_create": (ctypes.c_int, [ctypes.POINTER(vp), P, vp, ctypes.c_size_t]),
        "sph_destroy": (ctypes.c_int, [vp]),
        "sph_set_stream": (ctypes.c_int, [vp, vp]),
        "sph_set_params": (ctypes.c_int, [vp, P]),
        "sph_build_cells": (ctypes.c_int, [vp, PS]),
        "sph_density": (ctypes.c_int, [vp, PS]),
        "sph_forces": (ctypes.c_int, [vp, PS]),
        "sph_evaluate": (ctypes.c_int, [vp, PS]),
        "sph_upload_state": (ctypes.c_int, [vp, PS]),
        "sph_step": (ctypes.c_int, [vp, d, ctypes.POINTER(d)]),
        "sph_download_state": (ctypes.c_int, [vp, PS]),
        "sph_state_info": (ctypes.c_int, [vp, ctypes.POINTER(_Stats)]),
        "sph_neighbours": (ctypes.c_int, [vp, PS, i32, vp, vp, i64]),
        "sph_sync": (ctypes.c_int, [vp]),
        "sph_last_error": (ctypes.c_char_p, [vp]),
        "sph_device_bytes": (ctypes.c_size_t, [vp]),
        "sph_enable_kernel_timing": (ctypes.c_int, [vp, i32]),
        "sph_kernel_times": (ctypes.c_int, [vp, i32, ctypes.POINTER(d), ctypes.POINTER(i64)]),
        "sph_batch_density": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(PS), i32]),
        "sph_batch_forces": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(PS), i32]),
        "sph_batch_evaluate": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(PS), i32]),
        "sph_batch_step": (ctypes.c_int, [ctypes.POINTER(vp), i32, d]),
        "sph_batch_substep": (ctypes.c_int, [ctypes.POINTER(vp), i32]),
        "sph_capture_steps": (ctypes.c_int, [vp, d]),
        "sph_replay_steps": (ctypes.c_int, [vp]),
        "sph_plan_bytes": (ctypes.c_size_t, [P, i64]),
        "sph_evaluate_noalloc": (ctypes.c_int, [vp, PS]),
        "sph_noalloc_max_n": (i64, []),
        "sph_mfv_gradients": (ctypes.c_int, [vp, ctypes.POINTER(_MfvSet)]),
        "sph_substep": (ctypes.c_int, [vp]),
        "sph_server_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, i32]),
        "sph_server_submit": (ctypes.c_int, [vp, i32, ctypes.POINTER(_Request)]),
        "sph_server_wait": (i32, [vp, ctypes.POINTER(vp), i32, d]),
        "sph_server_release": (ctypes.c_int, [vp, i32]),
        "sph_server_slot_bytes": (ctypes.c_size_t, [vp, i32]),
        "sph_server_plan_bytes": (ctypes.c_size_t, [P, i64]),
        "sph_server_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def stats_dict(st: _Stats) -> dict:
    """sph_state_stats as a dict."""
    return {"time": st.time, "dt_last": st.dt_last, "dt_next": st.dt_next,
            "kinetic": st.kinetic, "thermal": st.thermal,
            "momentum": tuple(st.momentum), "steps": st.steps,
            "n_dens_pairs": st.n_dens_pairs, "n_force_pairs": st.n_force_pairs,
            "dens_pair_evals": st.dens_pair_evals, "force_pair_evals": st.force_pair_evals,
            "nr_iter_max": st.nr_iter_max, "walk_overflows": st.walk_overflows,
            "dens_leaf_visits": st.dens_leaf_visits, "dens_walks": st.dens_walks,
            "nr_iter_total": st.nr_iter_total,
            "dens_candidate_tests": st.dens_candidate_tests,
            "dens_box_tests": st.dens_box_tests,
            "force_candidate_tests": st.force_candidate_tests,
            "force_box_tests": st.force_box_tests,
            "density_walk_overflows": st.density_walk_overflows,
            "force_walk_overflows": st.force_walk_overflows,
            "dens_list_overflows": st.dens_list_overflows,
            "block_full_steps": st.block_full_steps, "block_substeps": st.block_substeps,
            "block_active": st.block_active, "block_updates": st.block_updates,
            "block_time": st.block_time, "block_dt_max": st.block_dt_max,
            "block_synchronised": st.block_synchronised}


@dataclass
class Params:
    """Method parameters (sph_params).  Defaults as sph_default_params."""
    eta: float = 1.2
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    ccfl: float = 0.2
    h_rtol: float = 1e-12
    h_max_iter: int = 50
    periodic: bool = True
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    precision: int = SPH_FP64
    leaf_size: int = 16
    alpha_ac: float = 0.0
    ac_signal: int = SPH_AC_WADSLEY
    av_switch: int = SPH_AV_NONE
    alpha_min: float = 0.1
    alpha_max: float = 1.0
    av_ell: float = 0.0
    block_lmax: int = 0
    block_lim: int = 2
    kernel: int = SPH_KERNEL_M4
    stage_leaves: int = 0       # launch shape: candidate leaves per LDS stage (0: 128/leaf)
    claim_leaves: int = 0       # launch shape: home leaves per claim (0: 1)

    @classmethod
    def from_setup(cls, setup: dict, **kw) -> "Params":
        keys = ("eta", "gamma", "alpha", "beta", "ccfl", "periodic", "lo", "hi", "alpha_ac",
                "ac_signal", "av_switch", "alpha_min", "alpha_max", "av_ell", "block_lmax",
                "block_lim", "kernel")
        return cls(**{k: setup[k] for k in keys if k in setup}, **kw)

    def c(self) -> _Params:
        p = _Params()
        p.eta, p.gamma, p.alpha_av, p.beta_av, p.c_cfl = (self.eta, self.gamma, self.alpha,
                                                          self.beta, self.ccfl)
        p.h_rtol, p.h_max_iter = self.h_rtol, int(self.h_max_iter)
        p.periodic = 1 if self.periodic else 0
        for k in range(3):
            p.box_lo[k] = float(self.lo[k])
            p.box_hi[k] = float(self.hi[k])
        p.precision = int(self.precision)
        p.leaf_size = int(self.leaf_size)
        p.alpha_ac = float(self.alpha_ac)
        p.ac_signal = int(self.ac_signal)
        p.av_switch = int(self.av_switch)
        p.alpha_min, p.alpha_max = float(self.alpha_min), float(self.alpha_max)
        p.av_ell = float(self.av_ell)
        p.block_lmax, p.block_lim = int(self.block_lmax), int(self.block_lim)
        p.kernel = int(self.kernel)
        p.stage_leaves, p.claim_leaves = int(self.stage_leaves), int(self.claim_leaves)
        return p


FIELDS_F64 = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "rho", "omega", "pressure", "cs",
              "ax", "ay", "az", "dudt", "vsig", "dt")
# optional arrays (after nngb/nforce in the C struct): only passed when present
FIELDS_OPT = ("alpha", "divv", "curlv", "level")
FIELDS_I32 = ("nngb", "nforce")


@dataclass
class Particles:
    """Device arrays of one particle set (caller index order)."""
    t: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.t["x"].numel())

    @classmethod
    def from_host(cls, arrays: dict, device="cuda", outputs: bool = True) -> "Particles":
        """Device copies of the inputs (and of the optional alpha when given),
        zeroed outputs.  divv / curlv are left out unless asked for with
        with_divv()."""
        t = {}
        for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "alpha"):
            if k in arrays:
                t[k] = torch.as_tensor(arrays[k], dtype=torch.float64).to(device).contiguous()
        n = t["x"].numel()
        if outputs:
            for k in FIELDS_F64:
                if k not in t:
                    t[k] = torch.zeros(n, dtype=torch.float64, device=device)
            for k in FIELDS_I32:
                t[k] = torch.zeros(n, dtype=torch.int32, device=device)
        return cls(t)

    def c(self, omit=()) -> _Particles:
        ps = _Particles()
        ps.n = self.n
        for k in FIELDS_F64 + FIELDS_I32 + FIELDS_OPT:
            v = self.t.get(k)
            if v is None or k in omit:
                setattr(ps, k, None)
                continue
            if not v.is_cuda:
                raise ValueError(f"{k} must be a GPU tensor")
            want = torch.int32 if k in FIELDS_I32 + ("level",) else torch.float64
            if v.dtype != want or not v.is_contiguous() or v.numel() != ps.n:
                raise ValueError(f"{k} must be a contiguous {want} tensor of {ps.n} elements")
            setattr(ps, k, v.data_ptr())
        return ps

    def with_level(self) -> "Particles":
        """Also request the time-step levels (sph_download_state)."""
        self.t["level"] = torch.zeros(self.n, dtype=torch.int32, device=self.t["x"].device)
        return self

    def with_divv(self) -> "Particles":
        """Also request the velocity divergence and curl outputs."""
        dev = self.t["x"].device
        for k in ("divv", "curlv"):
            self.t[k] = torch.zeros(self.n, dtype=torch.float64, device=dev)
        return self

    def host(self, *keys) -> dict:
        return {k: self.t[k].detach().cpu().numpy() for k in (keys or self.t.keys())}


class Context:
    """One sph_ctx bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, params: Params = None, stream: torch.cuda.Stream = None,
                 budget_bytes: int = 0):
        self.lib = load()
        self.params = params or Params()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._p = self.params.c()
        h = ctypes.c_void_p()
        rc = self.lib.sph_create(ctypes.byref(h), ctypes.byref(self._p),
                                 ctypes.c_void_p(self.stream.cuda_stream), int(budget_bytes))
        if rc != SPH_OK or not h.value:
            raise SphError(rc, "sph_create failed")
        self.h = h
        self._keep = None

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.sph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int, what: str):
        if rc != SPH_OK:
            msg = self.lib.sph_last_error(self.h)
            raise SphError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_params(self, params: Params):
        self.params = params
        self._p = params.c()
        self._check(self.lib.sph_set_params(self.h, ctypes.byref(self._p)), "sph_set_params")

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        self._check(self.lib.sph_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)),
                    "sph_set_stream")

    def build_cells(self, p: Particles):
        ps = p.c()
        self._check(self.lib.sph_build_cells(self.h, ctypes.byref(ps)), "sph_build_cells")

    def density(self, p: Particles, eos: bool = True):
        ps = p.c(omit=() if eos else ("pressure", "cs"))
        self._check(self.lib.sph_density(self.h, ctypes.byref(ps)), "sph_density")

    def forces(self, p: Particles):
        ps = p.c(omit=("pressure", "cs"))
        self._check(self.lib.sph_forces(self.h, ctypes.byref(ps)), "sph_forces")

    def evaluate(self, p: Particles):
        """Density (h solve) then forces: one full evaluation in one call, the
        set kept in sorted order on the device in between (sph_evaluate)."""
        ps = p.c()
        self._check(self.lib.sph_evaluate(self.h, ctypes.byref(ps)), "sph_evaluate")

    def evaluate_noalloc(self, p: Particles):
        """sph_evaluate without device allocation: the library's static
        scratch array holds every buffer (n <= sph_noalloc_max_n())."""
        ps = p.c()
        self._check(self.lib.sph_evaluate_noalloc(self.h, ctypes.byref(ps)), "sph_evaluate_noalloc")

    def mfv_gradients(self, x, y, z, h, fields=()) -> dict:
        """Meshless finite-volume geometry (sph_mfv_gradients) of device
        arrays x, y, z and the guess h (updated in place): number density,
        B = E^-1 (shape [n, 6]), condition number, gradients ([n, k, 3])."""
        n = int(x.numel())
        dev = x.device
        out = {"ndens": torch.zeros(n, dtype=torch.float64, device=dev),
               "nngb": torch.zeros(n, dtype=torch.int32, device=dev),
               "B": torch.zeros((6, n), dtype=torch.float64, device=dev),
               "cond": torch.zeros(n, dtype=torch.float64, device=dev),
               "grad": torch.zeros((max(len(fields), 1) * 3, n), dtype=torch.float64, device=dev)}
        s = _MfvSet()
        s.n = n
        s.x, s.y, s.z, s.h = x.data_ptr(), y.data_ptr(), z.data_ptr(), h.data_ptr()
        s.ndens, s.nngb, s.cond = (out["ndens"].data_ptr(), out["nngb"].data_ptr(),
                                   out["cond"].data_ptr())
        for k in range(6):
            s.B[k] = out["B"][k].data_ptr()
        s.nfields = len(fields)
        for k, f in enumerate(fields):
            s.f[k] = f.data_ptr()
            for a in range(3):
                s.grad[3 * k + a] = out["grad"][3 * k + a].data_ptr()
        self._check(self.lib.sph_mfv_gradients(self.h, ctypes.byref(s)), "sph_mfv_gradients")
        return out

    def density_then_forces(self, p: Particles):
        """The same evaluation as two calls, sph_density then sph_forces."""
        self.density(p)
        self.forces(p)

    def upload_state(self, p: Particles):
        ps = p.c()
        self._check(self.lib.sph_upload_state(self.h, ctypes.byref(ps)), "sph_upload_state")

    def substep(self):
        """One block time-step sub-step (sph_substep)."""
        self._check(self.lib.sph_substep(self.h), "sph_substep")

    def step(self, dt: float = 0.0):
        self._check(self.lib.sph_step(self.h, float(dt), None), "sph_step")

    def capture_steps(self, dt: float = 0.0):
        """Record two sph_step(dt) calls into a HIP graph (not executed)."""
        self._check(self.lib.sph_capture_steps(self.h, float(dt)), "sph_capture_steps")

    def replay_steps(self):
        """Launch the captured graph: two steps."""
        self._check(self.lib.sph_replay_steps(self.h), "sph_replay_steps")

    def download_state(self, p: Particles):
        ps = p.c()
        self._check(self.lib.sph_download_state(self.h, ctypes.byref(ps)), "sph_download_state")

    def state_info(self) -> dict:
        st = _Stats()
        self._check(self.lib.sph_state_info(self.h, ctypes.byref(st)), "sph_state_info")
        return stats_dict(st)

    def neighbours(self, p: Particles, mode: int, cap: int = None):
        """CSR lists at the given h -> (offsets int64[n+1], idx int32) on the device."""
        n = p.n
        dev = p.t["x"].device
        offsets = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        if cap is None:
            cap = max(1, 128 * n)
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        ps = p.c()
        rc = self.lib.sph_neighbours(self.h, ctypes.byref(ps), int(mode),
                                     ctypes.c_void_p(offsets.data_ptr()),
                                     ctypes.c_void_p(idx.data_ptr()), int(cap))
        if rc == SPH_ECAP:
            total = int(offsets[-1].item())
            return self.neighbours(p, mode, cap=total)
        self._check(rc, "sph_neighbours")
        return offsets, idx[:int(offsets[-1].item())]

    def sync(self):
        self._check(self.lib.sph_sync(self.h), "sph_sync")

    def sync_status(self) -> int:
        """sph_sync without raising: returns the status code."""
        return int(self.lib.sph_sync(self.h))

    def last_error(self) -> str:
        return self.lib.sph_last_error(self.h).decode()

    def device_bytes(self) -> int:
        return int(self.lib.sph_device_bytes(self.h))

    def enable_kernel_timing(self, on: bool = True, count_tests: bool = False):
        flags = (1 if on else 0) | (2 if count_tests else 0)
        self._check(self.lib.sph_enable_kernel_timing(self.h, flags), "timing")

    def kernel_times(self, which: int):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self.lib.sph_kernel_times(self.h, int(which), ctypes.byref(ms),
                                              ctypes.byref(cnt)), "sph_kernel_times")
        return ms.value, cnt.value

    def reset_kernel_times(self):
        for w in range(3):
            self._check(self.lib.sph_kernel_times(self.h, w, None, None), "sph_kernel_times")


def default_params_from_library() -> dict:
    p = _Params()
    load().sph_default_params(ctypes.byref(p))
    return {f: (tuple(getattr(p, f)) if f in ("box_lo", "box_hi") else getattr(p, f))
            for f, _ in _Params._fields_}


def _batch_arrays(ctxs, parts, omit):
    n = len(ctxs)
    hs = (ctypes.c_void_p * n)(*[c.h.value for c in ctxs])
    structs = [p.c(omit=omit) for p in parts]
    ptrs = (ctypes.POINTER(_Particles) * n)(*[ctypes.pointer(s) for s in structs])
    return hs, ptrs, structs


def _batch_check(ctxs, rc, what):
    if rc != SPH_OK:
        msgs = [c.last_error() for c in ctxs if c.last_error()]
        raise SphError(rc, f"{what}: {'; '.join(msgs)}")


def batch_density(ctxs, parts, eos: bool = True):
    """sph_batch_density over contexts sharing one stream."""
    lib = load()
    hs, ptrs, keep = _batch_arrays(ctxs, parts, () if eos else ("pressure", "cs"))
    _batch_check(ctxs, lib.sph_batch_density(hs, ptrs, len(ctxs)), "sph_batch_density")


def batch_forces(ctxs, parts):
    lib = load()
    hs, ptrs, keep = _batch_arrays(ctxs, parts, ("pressure", "cs"))
    _batch_check(ctxs, lib.sph_batch_forces(hs, ptrs, len(ctxs)), "sph_batch_forces")


def batch_evaluate(ctxs, parts):
    """sph_evaluate over many sets (sph_batch_evaluate)."""
    lib = load()
    hs, ptrs, keep = _batch_arrays(ctxs, parts, ())
    _batch_check(ctxs, lib.sph_batch_evaluate(hs, ptrs, len(ctxs)), "sph_batch_evaluate")


def batch_step(ctxs, dt: float = 0.0):
    lib = load()
    n = len(ctxs)
    hs = (ctypes.c_void_p * n)(*[c.h.value for c in ctxs])
    _batch_check(ctxs, lib.sph_batch_step(hs, n, float(dt)), "sph_batch_step")


def batch_substep(ctxs):
    """One block sub-step of each state, pair loops batched (sph_batch_substep)."""
    lib = load()
    n = len(ctxs)
    hs = (ctypes.c_void_p * n)(*[c.h.value for c in ctxs])
    _batch_check(ctxs, lib.sph_batch_substep(hs, n), "sph_batch_substep")


def plan_bytes(params: Params, n: int) -> int:
    """Device bytes a context needs for n particles (sph_plan_bytes)."""
    p = params.c()
    return int(load().sph_plan_bytes(ctypes.byref(p), int(n)))


def server_plan_bytes(params: Params, n: int) -> int:
    """Device bytes one executor slot needs for n particles (sph_server_plan_bytes)."""
    p = params.c()
    return int(load().sph_server_plan_bytes(ctypes.byref(p), int(n)))


class Server:
    """The library's request executor (sph_server_*): `slots` slots on the
    current device, each with its own HIP stream and context, driven by
    `threads` native worker threads (0: one per slot).  Requests are _Request
    structs that name host arrays; the caller keeps them (and the arrays)
    alive until wait() has returned their addresses."""

    def __init__(self, slots: int, threads: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        rc = self.lib.sph_server_create(ctypes.byref(h), int(slots), int(threads))
        if rc != SPH_OK or not h.value:
            raise SphError(rc, "sph_server_create failed")
        self.h = h
        self.slots = int(slots)
        self._done = (ctypes.c_void_p * 64)()

    def submit(self, slot: int, req: _Request):
        rc = self.lib.sph_server_submit(self.h, int(slot), ctypes.byref(req))
        if rc != SPH_OK:
            raise SphError(rc, f"sph_server_submit: slot {slot} is busy or the request is malformed")

    def wait(self, timeout: float) -> list:
        """Addresses (ctypes.addressof) of the requests completed within
        `timeout` seconds (0: poll; < 0: until one completes or none runs)."""
        k = self.lib.sph_server_wait(self.h, self._done, len(self._done), float(timeout))
        if k < 0:
            raise SphError(SPH_EINVAL, "sph_server_wait")
        return [int(self._done[i]) for i in range(k)]

    def release(self, slot: int):
        rc = self.lib.sph_server_release(self.h, int(slot))
        if rc != SPH_OK:
            raise SphError(rc, f"sph_server_release: slot {slot} is busy or out of range")

    def slot_bytes(self, slot: int) -> int:
        return int(self.lib.sph_server_slot_bytes(self.h, int(slot)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.sph_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_request(kind: int, arrays: dict, params: Params, nsteps: int = 0,
                 outputs: dict = None):
    """A _Request over host arrays: inputs x .. h from `arrays` (made
    contiguous float64), outputs into the numpy arrays of `outputs` (field
    name -> array of n values: float64 fields, int32 nngb / nforce).  Returns
    (request, arrays to keep alive until the request is returned)."""
    import numpy as np
    r = _Request()
    r.kind, r.nsteps = int(kind), int(nsteps)
    r.params = params.c()
    ins = [np.ascontiguousarray(arrays[k], dtype=np.float64) for k in FIELDS_F64[:NIN]]
    n = int(ins[0].size)
    r.n = n
    for i, a in enumerate(ins):
        if a.size != n:
            raise ValueError(f"{FIELDS_F64[i]} has {a.size} values, x has {n}")
        r.in_[i] = a.ctypes.data
    keep = list(ins)
    for k, a in (outputs or {}).items():
        want = np.int32 if k in FIELDS_I32 else np.float64
        if a.dtype != want or a.size != n or not a.flags.c_contiguous:
            raise ValueError(f"output {k} must be a contiguous {want.__name__} array of {n} values")
        if k in FIELDS_I32:
            r.iout[FIELDS_I32.index(k)] = a.ctypes.data
        else:
            r.out[FIELDS_F64.index(k)] = a.ctypes.data
        keep.append(a)
    return r, keep
