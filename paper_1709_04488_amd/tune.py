"""Autotuner for the pair-loop launch shape.

The knob is the leaf size G (8, 16 or 32 particles).  It fixes the whole
mapping of a pair loop onto the GPU: one wavefront per leaf of G home
particles, 64/G lanes per home particle, and 64/G candidate leaves (64
candidate particles) staged in LDS per step of the sweep.  Smaller leaves
give tighter candidate sets but more tree walks per particle; which wins
depends on N, on the precision of the pair arithmetic and on how clustered
the set is, so the tuner measures instead of guessing.

Requests are grouped into classes by (kind, precision, periodic, log2 N
rounded).  The first request of a class is timed at every leaf size (one
untimed call, then the best of `reps` timed calls, each a full density +
force evaluation on a private stream) and the fastest leaf size is kept for
the class; later requests of the class reuse it without measuring.  The
table can be saved to and loaded from a JSON file so a server starts tuned.
"""
from __future__ import annotations

import json
import math
import os
import time

LEAF_SIZES = (8, 16, 32)


def request_class(kind: str, precision: int, periodic: bool, n: int) -> str:
    """Class key of a request: kind, precision, boundary and log2 N rounded."""
    b = int(round(math.log2(max(n, 1))))
    return f"{kind}/p{int(precision)}/{'per' if periodic else 'open'}/n2^{b}"


class LeafTuner:
    """Leaf size per request class, measured on the first request of each class.

    `timer(arrays, setup, precision, leaf) -> seconds` times one evaluation;
    the default runs the HIP path (density + forces) on the GPU.  Tests pass a
    synthetic timer."""

    def __init__(self, sizes=LEAF_SIZES, reps: int = 2, path: str = None, timer=None):
        self.sizes = tuple(int(s) for s in sizes)
        self.reps = int(reps)
        self.path = path
        self.timer = timer or _gpu_timer(self.reps)
        self.table = {}          # class -> {"leaf": G, "seconds": {G: s}}
        if path and os.path.exists(path):
            self.load(path)

    # --- table ------------------------------------------------------------
    def load(self, path: str):
        with open(path) as f:
            data = json.load(f)
        self.table.update({k: v for k, v in data.items() if v.get("leaf") in self.sizes})

    def save(self, path: str = None):
        path = path or self.path
        if path:
            with open(path, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)

    # --- choice -----------------------------------------------------------
    def key(self, req) -> str:
        return request_class(req.kind, req.precision, bool(req.setup.get("periodic", True)), req.n)

    def choose(self, req) -> int:
        k = self.key(req)
        if k not in self.table:
            self.table[k] = self.measure(req.arrays, req.setup, req.precision)
            self.save()
        return int(self.table[k]["leaf"])

    __call__ = choose

    def measure(self, arrays, setup, precision: int) -> dict:
        secs = {}
        for g in self.sizes:
            secs[g] = float(self.timer(arrays, setup, precision, g))
        best = min(secs, key=lambda g: (secs[g], g))
        return {"leaf": int(best), "seconds": {str(g): s for g, s in secs.items()}}


def _gpu_timer(reps: int):
    def run(arrays, setup, precision, leaf):
        import torch

        from . import sph
        stream = torch.cuda.Stream()
        params = sph.Params.from_setup(setup, precision=precision, leaf_size=leaf)
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


def main(argv=None):
    import argparse

    from . import workloads as W
    ap = argparse.ArgumentParser(description="tune the leaf size on named workloads")
    ap.add_argument("--workload", default="c1", help="c0, c1, c2 or c1s<n_side>")
    ap.add_argument("--precision", type=int, default=None, help="0 FP64, 1 FP32-pair (default both)")
    ap.add_argument("--out", default=None, help="JSON table to update")
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    name = args.workload
    w = {"c0": W.config0, "c1": W.config1, "c2": W.config2}.get(name)
    w = w() if w else W.config1(n_side=int(name[3:]))
    tuner = LeafTuner(reps=args.reps, path=args.out)
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
