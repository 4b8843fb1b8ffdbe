"""Autotuner for the pair loops' launch shape.

Three separate choices of how the density and force loops map onto the GPU
(sph_params fields):

* leaf size G (8, 16 or 32 particles) -- the cell size.  One wavefront per
  leaf of G home particles with 64/G lanes each; smaller leaves give tighter
  candidate sets but more tree walks per particle.
* LDS stage depth (stage_leaves) -- candidate leaves staged in LDS per step
  of a sweep: the whole tile (128/G leaves) or half of it.  A shallower stage
  runs more, smaller test-and-flush rounds with denser hit masks; a deeper
  one fewer rounds.
* claim size (claim_leaves) -- home leaves a wavefront takes per atomic claim
  of the persistent loop (1 or 4): the wavefront-to-cell mapping.  Larger
  claims give a wave a run of neighbouring leaves (shared candidates in L2,
  fewer atomics) at the price of a coarser load balance at the end.

Which combination wins depends on N, the precision of the pair arithmetic
and how clustered the set is, so the tuner measures instead of guessing.
Requests are grouped into classes by (kind, precision, periodic, log2 N
rounded).  The first request of a class is timed by coordinate descent: every
leaf size at the default stage and claim, then the other stage depths at the
best leaf size, then the other claim sizes at the best (leaf, stage).  Later
requests of the class reuse the choice without measuring.  The table can be
saved to and loaded from a JSON file so a server starts tuned.

Two objectives:
* latency (default): one untimed call and the best of `reps` timed calls of
  a full density + force evaluation alone on a private stream;
* throughput (for serving): the device time of the pair loops per set when
  enough copies of the request share one batched launch to fill the GPU.
  A small set alone is fastest with the most parallel shape (G = 8: more
  waves, shorter chains per leaf), but when many sets share the GPU what
  counts is the GPU time each one occupies, which this measures.  (Timing
  a few concurrent copies by wall clock still rewards the parallel shape:
  they do not fill the GPU.)
"""
from __future__ import annotations

import json
import math
import os
import time

LEAF_SIZES = (8, 16, 32)
STAGES = ("full", "half")
CLAIMS = (1, 4)


def request_class(kind: str, precision: int, periodic: bool, n: int) -> str:
    """Class key of a request: kind, precision, boundary and log2 N rounded."""
    b = int(round(math.log2(max(n, 1))))
    return f"{kind}/p{int(precision)}/{'per' if periodic else 'open'}/n2^{b}"


def stage_leaves(leaf: int, stage: str) -> int:
    """sph_params.stage_leaves of a stage depth: 0 (the whole 128/G tile) or
    half of it."""
    if stage == "full":
        return 0
    if stage == "half":
        return max(1, 64 // int(leaf))
    raise ValueError(f"unknown stage depth {stage!r}")


def shape_key(shape: dict) -> str:
    return f"g{shape['leaf']}/{shape['stage']}/c{shape['claim']}"


def params_kw(shape: dict) -> dict:
    """sph.Params keyword arguments of a launch shape."""
    return {"leaf_size": int(shape["leaf"]),
            "stage_leaves": stage_leaves(shape["leaf"], shape["stage"]),
            "claim_leaves": int(shape["claim"])}


class LaunchTuner:
    """Launch shape per request class, measured on the first request of each
    class.

    `timer(arrays, setup, precision, shape) -> seconds` times one evaluation
    with shape = {"leaf": G, "stage": "full"|"half", "claim": C}; the default
    runs the HIP path (density + forces) on the GPU.  Tests pass a synthetic
    timer.  Calling the tuner on a request returns its leaf size (what memory
    planning needs); shape(req) returns the whole choice."""

    def __init__(self, sizes=LEAF_SIZES, stages=STAGES, claims=CLAIMS, reps: int = 2,
                 path: str = None, timer=None, objective: str = "latency"):
        self.sizes = tuple(int(s) for s in sizes)
        self.stages = tuple(stages)
        self.claims = tuple(int(c) for c in claims)
        self.reps = int(reps)
        self.path = path
        if objective not in ("latency", "throughput"):
            raise ValueError(f"unknown objective {objective!r}")
        self.objective = objective
        if timer is None:
            timer = _gpu_timer(self.reps) if objective == "latency" else _batch_timer(self.reps)
        self.timer = timer
        self.table = {}          # class -> {"leaf", "stage", "claim", "seconds": {shape: s}}
        if path and os.path.exists(path):
            self.load(path)

    # --- table ------------------------------------------------------------
    def _valid(self, v: dict) -> bool:
        return (v.get("leaf") in self.sizes and v.get("stage") in self.stages
                and v.get("claim") in self.claims)

    def load(self, path: str):
        with open(path) as f:
            data = json.load(f)
        self.table.update({k: v for k, v in data.items() if self._valid(v)})

    def save(self, path: str = None):
        path = path or self.path
        if path:
            with open(path, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)

    # --- choice -----------------------------------------------------------
    def key(self, req) -> str:
        k = request_class(req.kind, req.precision, bool(req.setup.get("periodic", True)), req.n)
        return k if self.objective == "latency" else k + "/throughput"

    def shape(self, req) -> dict:
        k = self.key(req)
        if k not in self.table:
            self.table[k] = self.measure(req.arrays, req.setup, req.precision)
            self.save()
        e = self.table[k]
        return {"leaf": int(e["leaf"]), "stage": e["stage"], "claim": int(e["claim"])}

    def choose(self, req) -> int:
        return self.shape(req)["leaf"]

    __call__ = choose

    def measure(self, arrays, setup, precision: int) -> dict:
        secs = {}

        def t(shape):
            k = shape_key(shape)
            if k not in secs:
                secs[k] = float(self.timer(arrays, setup, precision, dict(shape)))
            return secs[k]

        def best(cands):
            # ties go to the earlier candidate (smaller leaf, full stage, claim 1)
            return min(cands, key=lambda s: t(s))

        base = {"stage": self.stages[0], "claim": self.claims[0]}
        cur = best([{**base, "leaf": g} for g in self.sizes])
        cur = best([{**cur, "stage": s} for s in self.stages])
        cur = best([{**cur, "claim": c} for c in self.claims])
        return {**cur, "seconds": secs}


def _gpu_timer(reps: int):
    def run(arrays, setup, precision, shape):
        import torch

        from . import sph
        stream = torch.cuda.Stream()
        params = sph.Params.from_setup(setup, precision=precision, **params_kw(shape))
        with torch.cuda.stream(stream):
            ctx = sph.Context(params, stream=stream)
            p = sph.Particles.from_host(arrays)
            h0 = p.t["h"].clone()
            best = math.inf
            for r in range(reps + 1):
                p.t["h"].copy_(h0)
                stream.synchronize()
                t0 = time.perf_counter()
                ctx.evaluate(p)
                ctx.sync()
                dt = time.perf_counter() - t0
                if r > 0:
                    best = min(best, dt)
            ctx.close()
        return best
    return run


class _batch_timer:
    """Device seconds per set of the density and force loops when K copies of
    the request share one batched launch: K = ceil(2^18 / N) up to 64, so
    that small sets together give the launch enough leaves to fill the GPU.
    The time is that of the pair-loop kernels alone (HIP events around them,
    best of `reps` after an untimed call), divided by K.  The contexts are
    kept between timings (one stream) and take each shape's parameters."""

    TARGET_PARTICLES = 1 << 18
    MAX_COPIES = 64

    def __init__(self, reps: int):
        self.reps = int(reps)
        self.stream = None
        self.ctxs = []

    def __call__(self, arrays, setup, precision, shape):
        import numpy as np
        import torch

        from . import sph
        n = int(np.asarray(arrays["x"]).size)
        k = int(min(self.MAX_COPIES, max(1, math.ceil(self.TARGET_PARTICLES / max(n, 1)))))
        params = sph.Params.from_setup(setup, precision=precision, **params_kw(shape))
        if self.stream is None:
            self.stream = torch.cuda.Stream()
        best = math.inf
        with torch.cuda.stream(self.stream):
            while len(self.ctxs) < k:
                self.ctxs.append(sph.Context(params, stream=self.stream))
            ctxs = self.ctxs[:k]
            for c in ctxs:
                c.set_params(params)
            ctxs[0].enable_kernel_timing(True)
            parts = [sph.Particles.from_host(arrays) for _ in range(k)]
            h0 = parts[0].t["h"].clone()
            for r in range(self.reps + 1):
                for p in parts:
                    p.t["h"].copy_(h0)
                ctxs[0].sync()
                ctxs[0].reset_kernel_times()
                sph.batch_evaluate(ctxs, parts)
                ms = ctxs[0].kernel_times(0)[0] + ctxs[0].kernel_times(1)[0]
                if r > 0:
                    best = min(best, ms * 1e-3 / k)
            ctxs[0].enable_kernel_timing(False)
        return best

    def __del__(self):
        for c in self.ctxs:
            try:
                c.close()
            except Exception:
                pass


def main(argv=None):
    import argparse

    from . import workloads as W
    ap = argparse.ArgumentParser(description="tune the pair loops' launch shape on named workloads")
    ap.add_argument("--workload", default="c1", help="c0, c1, c2 or c1s<n_side>")
    ap.add_argument("--precision", type=int, default=None, help="0 FP64, 1 FP32-pair (default both)")
    ap.add_argument("--out", default=None, help="JSON table to update")
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    name = args.workload
    w = {"c0": W.config0, "c1": W.config1, "c2": W.config2}.get(name)
    w = w() if w else W.config1(n_side=int(name[3:]))
    tuner = LaunchTuner(reps=args.reps, path=args.out)
    precs = (0, 1) if args.precision is None else (args.precision,)
    out = {}
    for p in precs:
        k = request_class("evaluate", p, w.setup["periodic"], w.n)
        tuner.table[k] = tuner.measure(w.arrays, w.setup, p)
        out[k] = tuner.table[k]
    tuner.save()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
