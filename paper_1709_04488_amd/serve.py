"""Serving SPH requests on one GPU with continuous batching.

Two request kinds:
  * ``evaluate``  -- one density + force evaluation of a particle set;
  * ``integrate`` -- ``nsteps`` kick-drift-kick steps of a particle set kept
                     resident on the device, steps replayed from a captured
                     HIP graph.

The scheduler is plain Python and device-agnostic:
  * requests are admitted first-come first-served once they have arrived,
    a slot is free and their device memory fits the HBM budget;
  * admission is continuous: a request arriving while others run starts as
    soon as a slot and memory free up, without waiting for a batch boundary;
  * a slot keeps its context (and its device memory, grown to the largest
    set it served) between requests, so the budget counts slot capacity plus
    the particle arrays of running requests.
The executor does the device work.  ``GpuExecutor`` gives every slot its own
HIP stream, so the kernels of concurrent requests overlap on the device; in
``batched`` mode the evaluate requests admitted together are run through one
batched persistent launch instead.  ``FakeExecutor`` (CPU, simulated clock)
exercises the scheduler without a GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import heapq
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

GIB = 1 << 30


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the run
    kind: str                      # "evaluate" or "integrate"
    arrays: dict                   # host float64 arrays x..h
    setup: dict
    precision: int = 0             # 0 FP64, 1 FP32-pair
    nsteps: int = 0

    @property
    def n(self) -> int:
        return int(self.arrays["x"].size)


@dataclass
class Record:
    rid: int
    n: int
    kind: str
    precision: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    slot: int = -1
    interactions: int = 0
    error: str = ""
    outputs: dict = field(default_factory=dict)
    info: dict = field(default_factory=dict)
    host_seconds: tuple = ()       # native executor: the slot thread's time, by phase

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# ----------------------------------------------------------------------------
# clocks
# ----------------------------------------------------------------------------
class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.05))


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float):
        self.t = max(self.t, t)


# ----------------------------------------------------------------------------
# scheduler
# ----------------------------------------------------------------------------
class Scheduler:
    def __init__(self, executor, budget_bytes: int, max_slots: int, clock=None, progress=None):
        self.ex = executor
        self.progress = progress                  # callable(done, total) or None
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock or WallClock()
        self.slot_cap = [0] * self.max_slots      # particles each slot's context can hold
        self.slot_leaf = [0] * self.max_slots     # largest leaf size its context has run
        self.slot_busy = [False] * self.max_slots
        self.array_bytes = {}                     # running rid -> bytes of its particle arrays
        self.peak_bytes = 0
        self.events = []                          # (time, what, rid)

    # memory currently held: slot capacities + arrays of running requests
    def used_bytes(self) -> int:
        return (sum(self.ex.slot_bytes(c, g) for c, g in zip(self.slot_cap, self.slot_leaf)) +
                sum(self.array_bytes.values()))

    def _fit(self, req: Request):
        """Free slot for req and the extra bytes admitting it costs, or None."""
        used = self.used_bytes()
        best = None
        for s in range(self.max_slots):
            if self.slot_busy[s]:
                continue
            cap = self.slot_cap[s]
            # the slot's context grows to the request's n; its scratch keeps
            # the size of the largest leaf size it has run
            leaf = max(self.slot_leaf[s], self.ex.leaf_of(req))
            extra = (self.ex.slot_bytes(max(cap, req.n), leaf) -
                     self.ex.slot_bytes(cap, self.slot_leaf[s]))
            extra += self.ex.array_bytes(req)
            if used + extra <= self.budget:
                # prefer the slot that grows least, then the smallest capacity
                key = (extra, cap)
                if best is None or key < best[0]:
                    best = (key, s, extra)
        return None if best is None else (best[1], best[2])

    def _release_idle(self, req: Request):
        """Free the capacity of idle slots, largest first, until req fits.
        Slot capacities only grow while slots are reused, so without this an
        idle server whose slots hold most of the budget could never admit the
        next request."""
        idle = sorted((s for s in range(self.max_slots)
                       if not self.slot_busy[s] and self.slot_cap[s] > 0),
                      key=lambda s: -self.slot_cap[s])
        for s in idle:
            self.ex.release(s)
            self.slot_cap[s] = 0
            self.slot_leaf[s] = 0
            self.events.append((self.clock.now(), "release", s))
            fit = self._fit(req)
            if fit is not None:
                return fit
        return None

    def _never_fits(self, req: Request) -> bool:
        return self.ex.slot_bytes(req.n, self.ex.leaf_of(req)) + self.ex.array_bytes(req) > self.budget

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        recs = {r.rid: Record(r.rid, r.n, r.kind, r.precision, r.arrival) for r in pending}
        queue = []
        running = {}
        k = 0
        while k < len(pending) or queue or running:
            now = self.clock.now()
            while k < len(pending) and pending[k].arrival <= now:
                queue.append(pending[k])
                k += 1
            # admit in arrival order; a request that can never fit is rejected
            started = []
            while queue:
                req = queue[0]
                if self._never_fits(req):
                    queue.pop(0)
                    recs[req.rid].error = "exceeds HBM budget"
                    recs[req.rid].done = now
                    continue
                fit = self._fit(req) or self._release_idle(req)
                if fit is None:
                    break
                slot, _ = fit
                queue.pop(0)
                self.slot_busy[slot] = True
                self.slot_cap[slot] = max(self.slot_cap[slot], req.n)
                self.slot_leaf[slot] = max(self.slot_leaf[slot], self.ex.leaf_of(req))
                self.array_bytes[req.rid] = self.ex.array_bytes(req)
                self.peak_bytes = max(self.peak_bytes, self.used_bytes())
                rec = recs[req.rid]
                rec.admitted = now
                rec.slot = slot
                started.append((req, slot))
                self.events.append((now, "admit", req.rid))
            if started:
                handles = self.ex.start(started)
                for (req, slot), h in zip(started, handles):
                    running[req.rid] = (req, slot, h)
            # completions
            finished = [rid for rid, (req, slot, h) in running.items() if self.ex.poll(h)]
            for rid in finished:
                req, slot, h = running.pop(rid)
                rec = recs[rid]
                try:
                    out = self.ex.finish(h)
                    rec.outputs = out.get("outputs", {})
                    rec.interactions = int(out.get("interactions", 0))
                    rec.info = out.get("info", {})
                    rec.host_seconds = tuple(out.get("host_seconds", ()))
                except Exception as e:  # reported per request, the server keeps going
                    rec.error = str(e)
                rec.done = self.clock.now()
                self.slot_busy[slot] = False
                self.array_bytes.pop(rid, None)
                self.events.append((rec.done, "done", rid))
                if self.progress:
                    self.progress(sum(1 for r in recs.values() if not math.isnan(r.done)), len(recs))
            if not started and not finished:
                nxt = pending[k].arrival if k < len(pending) else math.inf
                self.ex.wait(self.clock, nxt)
        return [recs[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(recs, makespan: float) -> dict:
    ok = [r for r in recs if not r.error]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    inter = sum(r.interactions for r in ok)
    return {"requests": len(recs), "completed": len(ok), "errors": len(recs) - len(ok),
            "makespan_s": makespan, "throughput_interactions_per_s": inter / makespan if makespan > 0 else 0.0,
            "requests_per_s": len(ok) / makespan if makespan > 0 else 0.0,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "latency_max_ms": float(lat.max() * 1e3),
            **_host_phases(ok)}


def _host_phases(recs) -> dict:
    """Native executor: the slot threads' summed time per phase of a request."""
    hs = [r.host_seconds for r in recs if r.host_seconds]
    if not hs:
        return {}
    tot = np.sum(np.array(hs), axis=0)
    return {"slot_thread_seconds": dict(zip(("stage_inputs", "enqueue", "in_flight",
                                             "write_outputs"), map(float, tot)))}


# ----------------------------------------------------------------------------
# executors
# ----------------------------------------------------------------------------
class FakeExecutor:
    """Simulated device: a request takes cost(req) seconds once started; up to
    `lanes` requests progress at once (processor sharing is not modelled)."""

    def __init__(self, clock, cost, bytes_per_particle: int = 500, fixed: int = 1 << 20):
        self.clock = clock
        self.cost = cost
        self.bpp = bytes_per_particle
        self.fixed = fixed
        self.starts = []
        self.active = {}
        self.released = []

    def slot_bytes(self, cap: int, leaf: int = 16) -> int:
        return 0 if cap == 0 else self.fixed + self.bpp * cap

    def leaf_of(self, req: Request) -> int:
        return 16

    def array_bytes(self, req: Request) -> int:
        return 168 * req.n

    def start(self, items):
        hs = []
        for req, slot in items:
            t = self.clock.now()
            self.starts.append((t, req.rid, slot))
            h = {"req": req, "end": t + self.cost(req)}
            self.active[req.rid] = h["end"]
            hs.append(h)
        return hs

    def poll(self, h) -> bool:
        return self.clock.now() >= h["end"]

    def finish(self, h):
        self.active.pop(h["req"].rid, None)
        return {"interactions": 100 * h["req"].n}

    def release(self, slot: int):
        self.released.append(slot)

    def wait(self, clock, next_arrival: float):
        # advance to the next event: an arrival or the earliest completion
        t = min([next_arrival] + list(self.active.values()))
        clock.sleep_until(t if math.isfinite(t) else clock.now() + 1e-3)


def _request_params(sph, leaf_for, req: Request):
    """sph.Params of a request: its setup and precision, with the launch shape
    a tuner chooses (leaf size, stage depth, claim size) or the leaf size a
    plain function gives."""
    shape_of = getattr(leaf_for, "shape", None)
    if shape_of is not None:
        from .tune import params_kw
        return sph.Params.from_setup(req.setup, precision=req.precision, **params_kw(shape_of(req)))
    return sph.Params.from_setup(req.setup, precision=req.precision, leaf_size=leaf_for(req))


class _Slot:
    def __init__(self, idx, stream, ctx):
        self.idx = idx
        self.stream = stream
        self.ctx = ctx
        self.pinned = {}      # name -> reusable pinned host buffer (grown on demand)

    def host_buffer(self, torch, name: str, count: int, dtype):
        """Pinned host staging of at least `count` elements, reused by every
        request of this slot (a slot runs one request at a time, and its
        copies finish before the next request starts)."""
        buf = self.pinned.get(name)
        if buf is None or buf.numel() < count:
            buf = torch.empty(max(count, 1), dtype=dtype).pin_memory()
            self.pinned[name] = buf
        return buf[:count]


class GpuExecutor:
    """Requests on the MI355X through the sph C ABI, one HIP stream per slot."""

    OUT_EVAL = ("h", "rho", "omega", "pressure", "cs", "ax", "ay", "az", "dudt", "vsig", "dt",
                "nngb", "nforce")

    def __init__(self, max_slots: int, mode: str = "streams", leaf_for=None, keep_outputs=False,
                 download=True, threads=True):
        import torch

        from . import sph
        self.torch = torch
        self.sph = sph
        self.mode = mode
        # a request is done when its results are in host memory (download);
        # keep_outputs also stores them in the request's record
        self.keep_outputs = keep_outputs
        self.download = download or keep_outputs
        self.leaf_for = leaf_for or (lambda req: 16)
        self.shared = torch.cuda.Stream()
        self.slots = []
        for s in range(max_slots):
            stream = self.shared if mode == "batched" else torch.cuda.Stream()
            self.slots.append(_Slot(s, stream, None))
        # streams mode: one worker thread per slot carries a request from the
        # upload through its kernels to the results in host memory, so host
        # copies and launches of different slots overlap (copies and C calls
        # run without the interpreter lock); each slot's context is used by
        # one thread at a time
        self.pool = None
        self.inflight = set()   # worker-thread futures not yet finished
        if threads and mode == "streams":
            from concurrent.futures import ThreadPoolExecutor
            self.pool = ThreadPoolExecutor(max_workers=max_slots)

    def close(self):
        if self.pool is not None:
            self.pool.shutdown(wait=True)
            self.pool = None

    def params(self, req: Request):
        return _request_params(self.sph, self.leaf_for, req)

    def slot_bytes(self, cap: int, leaf: int = 16) -> int:
        return 0 if cap == 0 else self.sph.plan_bytes(self.sph.Params(leaf_size=leaf or 16), cap)

    def leaf_of(self, req: Request) -> int:
        return int(self.leaf_for(req))

    def array_bytes(self, req: Request) -> int:
        return req.n * 8 * 19 + req.n * 4 * 2

    def _ctx(self, slot: _Slot, req: Request):
        if slot.ctx is None:
            slot.ctx = self.sph.Context(self.params(req), stream=slot.stream)
        else:
            slot.ctx.set_params(self.params(req))
        return slot.ctx

    # the inputs are the first 9 of the 19 FP64 fields (x .. h), the
    # evaluation's FP64 outputs the last 11 (h .. dt): one copy each way
    N_IN = 9

    def _upload(self, req: Request, slot: _Slot):
        """All fields of a request in one device block (19 FP64 rows, 2 int32
        rows); the 9 input rows arrive in one copy from the slot's pinned
        staging buffer."""
        torch = self.torch
        F = self.sph.FIELDS_F64
        n = req.n
        host = slot.host_buffer(torch, "in", self.N_IN * n, torch.float64).view(self.N_IN, n)
        for i, k in enumerate(F[:self.N_IN]):
            host[i].copy_(torch.from_numpy(np.ascontiguousarray(req.arrays[k], dtype=np.float64)))
        with torch.cuda.stream(slot.stream):
            dev = torch.empty((len(F), n), dtype=torch.float64, device="cuda")
            idev = torch.empty((len(self.sph.FIELDS_I32), n), dtype=torch.int32, device="cuda")
            dev[:self.N_IN].copy_(host, non_blocking=True)
        t = {k: dev[i] for i, k in enumerate(F)}
        t.update({k: idev[i] for i, k in enumerate(self.sph.FIELDS_I32)})
        return self.sph.Particles(t), dev, idev

    def _results(self, h) -> dict:
        """The evaluation's outputs in host memory (two copies through the
        slot's pinned buffers); numpy views of those buffers unless kept."""
        torch = self.torch
        slot, dev, idev = h["slot"], h["dev"], h["idev"]
        n = dev.shape[1]
        first = self.N_IN - 1                      # h: the last input, the first output
        outs = self.sph.FIELDS_F64[first:]
        hf = slot.host_buffer(torch, "out", len(outs) * n, torch.float64).view(len(outs), n)
        hi = slot.host_buffer(torch, "iout", idev.numel(), torch.int32).view(idev.shape[0], n)
        with torch.cuda.stream(slot.stream):
            hf.copy_(dev[first:], non_blocking=True)
            hi.copy_(idev, non_blocking=True)
        slot.stream.synchronize()
        res = {k: hf[i].numpy() for i, k in enumerate(outs)}
        res.update({k: hi[i].numpy() for i, k in enumerate(self.sph.FIELDS_I32)})
        return {k: res[k] for k in self.OUT_EVAL}

    def _zeros(self, n: int, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            t = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in self.sph.FIELDS_F64}
            for k in self.sph.FIELDS_I32:
                t[k] = torch.zeros(n, dtype=torch.int32, device="cuda")
        return self.sph.Particles(t)

    def _prepare(self, req: Request, slot: _Slot) -> dict:
        ctx = self._ctx(slot, req)
        p, dev, idev = self._upload(req, slot)
        return {"req": req, "slot": slot, "ctx": ctx, "p": p, "dev": dev, "idev": idev,
                "event": self.torch.cuda.Event()}

    def _launch(self, h):
        """Enqueue one request's work on its slot's stream."""
        torch, req, ctx, p, slot = self.torch, h["req"], h["ctx"], h["p"], h["slot"]
        with torch.cuda.stream(slot.stream):
            if req.kind == "evaluate":
                ctx.evaluate(p)
            elif ctx.params.block_lmax > 0:
                # block time-steps: sub-steps until nsteps level-0 steps are
                # done (the clock is read between them), their pairs summed
                ctx.upload_state(p)
                h["block_pairs"] = 0
                while ctx.state_info()["block_full_steps"] < req.nsteps:
                    ctx.substep()
                    i = ctx.state_info()
                    h["block_pairs"] += i["n_dens_pairs"] + i["n_force_pairs"]
            else:
                ctx.upload_state(p)
                ctx.capture_steps(0.0)
                for _ in range(req.nsteps // 2):
                    ctx.replay_steps()
                if req.nsteps % 2:
                    ctx.step(0.0)
        h["event"].record(slot.stream)

    def _block_batch(self, hs):
        """Block integration requests admitted together (batched mode, one
        shared stream): every state advances by sph_batch_substep, each on its
        own clock, its pair loops launched with the others'; a state leaves the
        batch once its level-0 steps are done."""
        torch = self.torch
        with torch.cuda.stream(self.shared):
            for h in hs:
                h["ctx"].upload_state(h["p"])
                h["block_pairs"] = 0
            live = [h for h in hs if h["req"].nsteps > 0]
            while live:
                self.sph.batch_substep([h["ctx"] for h in live])
                nxt = []
                for h in live:
                    i = h["ctx"].state_info()
                    h["block_pairs"] += i["n_dens_pairs"] + i["n_force_pairs"]
                    if i["block_full_steps"] < h["req"].nsteps:
                        nxt.append(h)
                live = nxt
            ev = torch.cuda.Event()
            ev.record(self.shared)
        for h in hs:
            h["event"] = ev

    def _serve_one(self, req: Request, slot: _Slot) -> dict:
        """A worker thread's whole request: upload, kernels, results on the host."""
        h = self._prepare(req, slot)
        self._launch(h)
        return self._finish(h)

    def start(self, items):
        if self.pool is not None:
            hs = [{"req": req, "future": self.pool.submit(self._serve_one, req, self.slots[sidx])}
                  for req, sidx in items]
            self.inflight.update(h["future"] for h in hs)
            return hs
        torch = self.torch
        handles = [None] * len(items)
        batch = []
        blocks = []
        for k, (req, sidx) in enumerate(items):
            h = self._prepare(req, self.slots[sidx])
            if req.kind == "evaluate" and self.mode == "batched":
                batch.append(h)
            elif self.mode == "batched" and h["ctx"].params.block_lmax > 0:
                blocks.append(h)
            else:
                self._launch(h)
            handles[k] = h
        if blocks:
            self._block_batch(blocks)
        if batch:
            self.sph.batch_evaluate([h["ctx"] for h in batch], [h["p"] for h in batch])
            ev = torch.cuda.Event()
            ev.record(self.shared)
            for h in batch:
                h["event"] = ev
        return handles

    def poll(self, h) -> bool:
        if "future" in h:
            return h["future"].done()
        return h["event"].query()

    def finish(self, h):
        if "future" in h:
            self.inflight.discard(h["future"])
            return h["future"].result()
        return self._finish(h)

    def _finish(self, h):
        ctx, p, req = h["ctx"], h["p"], h["req"]
        rc = ctx.sync_status()
        if rc != self.sph.SPH_OK:
            raise self.sph.SphError(rc, ctx.last_error())
        info = ctx.state_info()
        out = {"info": info}
        if req.kind == "evaluate":
            out["interactions"] = info["n_dens_pairs"] + info["n_force_pairs"]
            if self.download:
                res = self._results(h)
                if self.keep_outputs:
                    out["outputs"] = {k: v.copy() for k, v in res.items()}
        else:
            out["interactions"] = (h["block_pairs"] if "block_pairs" in h and req.nsteps > 0 else
                                   (info["n_dens_pairs"] + info["n_force_pairs"]) * max(req.nsteps, 1))
            q = self._zeros(req.n, h["slot"].stream)
            ctx.download_state(q)
            ctx.sync()
            if self.download:
                res = q.host("x", "y", "z", "vx", "vy", "vz", "u", "h")
                if self.keep_outputs:
                    out["outputs"] = res
        h["p"] = h["dev"] = h["idev"] = None
        return out

    def release(self, slot: int):
        sl = self.slots[slot]
        if sl.ctx is not None:
            sl.ctx.close()
            sl.ctx = None

    def wait(self, clock, next_arrival: float):
        """Until a running request completes or the next one arrives.  With
        worker threads the wait wakes on the first completion itself;
        otherwise the device events are polled every 0.2 ms."""
        if self.inflight:
            from concurrent.futures import FIRST_COMPLETED
            from concurrent.futures import wait as wait_futures
            t = next_arrival - clock.now() if math.isfinite(next_arrival) else 0.05
            wait_futures(self.inflight, timeout=max(0.0, min(t, 0.05)), return_when=FIRST_COMPLETED)
            return
        time.sleep(0.0002)


class NativeExecutor:
    """Requests through the library's own executor (sph_server_*): each slot's
    native worker thread stages the inputs, copies them to the device, runs
    the request on the slot's stream and writes the outputs into host arrays,
    so the interpreter only admits requests and collects them.  A slot's
    device memory is its context plus its particle arrays, both kept at the
    slot's capacity (counted in slot_bytes, none per request)."""

    OUT_EVAL = GpuExecutor.OUT_EVAL
    OUT_INTEGRATE = ("x", "y", "z", "vx", "vy", "vz", "u", "h")

    def __init__(self, max_slots: int, leaf_for=None, keep_outputs=False, download=True,
                 threads: int = 0):
        from . import sph
        self.sph = sph
        self.server = sph.Server(max_slots, threads)
        self.leaf_for = leaf_for or (lambda req: 16)
        self.keep_outputs = keep_outputs
        self.download = download or keep_outputs
        self.host = [dict() for _ in range(max_slots)]   # reusable host outputs per slot
        self.pending = {}                                # request address -> handle

    def close(self):
        self.server.close()

    def params(self, req: Request):
        return _request_params(self.sph, self.leaf_for, req)

    def slot_bytes(self, cap: int, leaf: int = 16) -> int:
        return 0 if cap == 0 else self.sph.server_plan_bytes(self.sph.Params(leaf_size=leaf or 16), cap)

    def leaf_of(self, req: Request) -> int:
        return int(self.leaf_for(req))

    def array_bytes(self, req: Request) -> int:
        return 0

    def _outputs(self, slot: int, req: Request) -> dict:
        if not self.download:
            return {}
        names = self.OUT_EVAL if req.kind == "evaluate" else self.OUT_INTEGRATE
        n = req.n
        out = {}
        for k in names:
            dt = np.int32 if k in self.sph.FIELDS_I32 else np.float64
            if self.keep_outputs:
                out[k] = np.empty(n, dtype=dt)
                continue
            buf = self.host[slot].get(k)
            if buf is None or buf.size < n:
                buf = np.empty(max(n, 1), dtype=dt)
                self.host[slot][k] = buf
            out[k] = buf[:n]
        return out

    def start(self, items):
        hs = []
        for req, slot in items:
            kind = (self.sph.SPH_REQUEST_EVALUATE if req.kind == "evaluate"
                    else self.sph.SPH_REQUEST_INTEGRATE)
            outs = self._outputs(slot, req)
            r, keep = self.sph.make_request(kind, req.arrays, self.params(req), req.nsteps, outs)
            h = {"req": req, "r": r, "keep": keep, "outputs": outs, "done": False}
            addr = ctypes.addressof(r)
            self.pending[addr] = h
            try:
                self.server.submit(slot, r)
            except Exception:
                del self.pending[addr]
                raise
            hs.append(h)
        return hs

    def _collect(self, timeout: float):
        for addr in self.server.wait(timeout):
            self.pending.pop(addr)["done"] = True

    def poll(self, h) -> bool:
        if not h["done"]:
            self._collect(0.0)
        return h["done"]

    def finish(self, h):
        r, req = h["r"], h["req"]
        h["keep"] = None
        if r.status != self.sph.SPH_OK:
            raise self.sph.SphError(r.status, r.error.decode(errors="replace"))
        out = {"info": self.sph.stats_dict(r.info), "interactions": int(r.interactions),
               "host_seconds": tuple(r.host_seconds)}
        if self.keep_outputs:
            out["outputs"] = h["outputs"]
        return out

    def release(self, slot: int):
        self.server.release(slot)

    def wait(self, clock, next_arrival: float):
        """Until a running request completes (the library wakes the wait) or
        the next one arrives."""
        t = next_arrival - clock.now() if math.isfinite(next_arrival) else 0.05
        if self.pending:
            self._collect(max(0.0, min(t, 0.05)))
        else:
            clock.sleep_until(next_arrival if math.isfinite(next_arrival) else clock.now() + 1e-3)


# ----------------------------------------------------------------------------
# the two served workloads
# ----------------------------------------------------------------------------
def evaluate_requests(count: int, rate: float, seed: int = 3, n_max_side: int = None):
    """Serving mix: jittered-lattice boxes, N log-uniform in [1e3, 2e5]
    snapped to n^3, FP64 or FP32-pair with probability 1/2, Poisson
    arrivals at `rate` per second (rate = inf: all at t = 0)."""
    from . import workloads as W
    spec = W.config3_requests(count, seed=seed)
    rng = np.random.default_rng(seed + 7)
    t = 0.0
    reqs = []
    for rid, (side, prec, wseed) in enumerate(spec):
        if n_max_side:
            side = min(side, n_max_side)
        w = W.jittered_lattice(side, seed=wseed)
        if math.isfinite(rate):
            t += rng.exponential(1.0 / rate)
        reqs.append(Request(rid, t if math.isfinite(rate) else 0.0, "evaluate", w.arrays, w.setup,
                            precision=int(prec)))
    return reqs


def integrate_requests(count: int, nsteps: int, rate: float = math.inf, seed: int = 4,
                       n_max_side: int = None, precision: int = 1, block: bool = False):
    """Served integration: blob-in-lattice boxes, N log-uniform in [1e4, 1e6]
    snapped to n^3, FP32-pair pair arithmetic with FP64 state.  block: every
    request on hierarchical block time-steps (levels down to 2^-20 of the
    level-0 step, limiter 2 levels), nsteps then counting level-0 steps."""
    from . import workloads as W
    spec = W.config4_requests(count, seed=seed)
    rng = np.random.default_rng(seed + 7)
    t = 0.0
    reqs = []
    for rid, (side, wseed) in enumerate(spec):
        if n_max_side:
            side = min(side, n_max_side)
        w = W.blob_in_lattice(side, seed=wseed)
        if math.isfinite(rate):
            t += rng.exponential(1.0 / rate)
        setup = {**w.setup, "block_lmax": 20, "block_lim": 2} if block else w.setup
        reqs.append(Request(rid, t if math.isfinite(rate) else 0.0, "integrate", w.arrays, setup,
                            precision=precision, nsteps=nsteps))
    return reqs


def _progress(done: int, total: int):
    if done == total or done % 16 == 0:
        print(f"# served {done}/{total}", file=sys.stderr, flush=True)


def serve(reqs, budget: int, slots: int, mode: str, leaf_for=None, keep_outputs=False,
          progress=False, download=True, threads=True, native_threads: int = 0):
    """Serve `reqs`; a request completes when its results are in host memory
    (download=False stops at the device, for measurements of that part).
    threads: in streams mode, one worker thread per slot; native_threads: the
    native executor's worker threads (0: one per slot)."""
    import torch
    if mode == "native":
        ex = NativeExecutor(slots, leaf_for=leaf_for, keep_outputs=keep_outputs, download=download,
                            threads=native_threads)
    else:
        ex = GpuExecutor(slots, mode=mode, leaf_for=leaf_for, keep_outputs=keep_outputs,
                         download=download, threads=threads)
    sched = Scheduler(ex, budget, slots, WallClock(), progress=_progress if progress else None)
    t0 = sched.clock.now()
    try:
        recs = sched.run(reqs)
    finally:
        ex.close()
    torch.cuda.synchronize()
    makespan = max(r.done for r in recs) - t0
    out = summarize(recs, makespan)
    out["peak_bytes"] = sched.peak_bytes
    return recs, out


def serving_tuner(reqs, budget: int, slots: int, tune_table: str = None):
    """Launch-shape tuner for a served workload: each request class tuned for
    the GPU time it occupies (many requests share the GPU), among the leaf
    sizes whose slot footprint at the largest request fits the per-slot share
    of the HBM budget.  A larger leaf size enlarges a slot's candidate-list
    scratch (G = 32: twice that of G = 16); where that pushes slots past their
    share, the budget admits fewer requests at once, which costs more than
    the shape gains."""
    from . import sph
    from .tune import LEAF_SIZES, LaunchTuner
    n_max = max((r.n for r in reqs), default=1)
    share = budget // max(int(slots), 1)
    sizes = tuple(g for g in LEAF_SIZES
                  if sph.server_plan_bytes(sph.Params(leaf_size=g), n_max) <= share)
    return LaunchTuner(sizes=sizes or (min(LEAF_SIZES),), path=tune_table, objective="throughput")


def run_served(workload: str = "evaluate", requests: int = 512, steps: int = 200,
               budget_gib: float = None, slots: int = 3, mode: str = "native",
               load: float = 0.8, max_side: int = None, leaf="auto", tune_table: str = None,
               threads: bool = True, progress: bool = True, saturated_only: bool = False,
               repeat: int = 1, block: bool = False) -> dict:
    """Serve one of the two workloads and summarise it.  evaluate: a closed
    burst (every request at t = 0) gives the saturated capacity, then Poisson
    arrivals at `load` times that rate (saturated_only: the burst alone);
    integrate: `requests` resident integrations of `steps` KDK steps each
    (block: `steps` level-0 steps of block time-steps each).
    Every request class is tuned before the timed runs when leaf is "auto".
    repeat: serve the burst that many times, 0.2 s apart (the last pass is
    reported; a trace can tell the passes apart by the pause)."""
    gib = budget_gib if budget_gib else (1.0 if workload == "evaluate" else 16.0)
    budget = int(gib * GIB)

    def pretune(reqs):
        nonlocal leaf_for
        if leaf == "auto":
            leaf_for = serving_tuner(reqs, budget, slots, tune_table)
            for r in reqs:
                leaf_for(r)
        else:
            g = int(leaf)
            leaf_for = lambda req: g  # noqa: E731

    leaf_for = None
    if workload == "evaluate":
        burst = evaluate_requests(requests, math.inf, n_max_side=max_side)
        pretune(burst)
        for k in range(max(int(repeat), 1)):
            if k:
                time.sleep(0.2)
            _, closed = serve(burst, budget, slots, mode, leaf_for=leaf_for, progress=progress,
                              threads=threads)
        res = {"workload": "evaluate", "mode": mode, "slots": slots, "leaf": leaf,
               "budget_bytes": budget, "saturated": closed}
        if not saturated_only:
            rate = load * closed["requests_per_s"]
            reqs = evaluate_requests(requests, rate, n_max_side=max_side)
            _, opened = serve(reqs, budget, slots, mode, leaf_for=leaf_for, progress=progress,
                              threads=threads)
            res.update({"arrival_rate_per_s": rate, "poisson": opened})
    else:
        reqs = integrate_requests(requests, steps, n_max_side=max_side, block=block)
        pretune(reqs)
        recs, out = serve(reqs, budget, slots, mode, leaf_for=leaf_for, progress=progress,
                          threads=threads)
        ok = [r for r in recs if not r.error]
        nsteps = sum(r.info.get("steps", 0) for r in ok)
        per_step = [r.latency / max(steps, 1) * 1e3 for r in ok] or [0.0]
        res = {"workload": "integrate", "mode": mode, "slots": slots, "leaf": leaf,
               "budget_bytes": budget, "steps_per_request": steps, "result": out,
               "steps_total": nsteps,
               "per_step_latency_p50_ms": float(np.percentile(per_step, 50)),
               "per_step_latency_p99_ms": float(np.percentile(per_step, 99))}
        if block:
            upd = sum(r.info.get("block_updates", 0) for r in ok)
            res.update({"block_time_steps": True,
                        "substeps_total": sum(r.info.get("block_substeps", 0) for r in ok),
                        "particle_updates_total": upd,
                        "particles_total": sum(r.n for r in ok),
                        "particle_updates_per_s": upd / max(out["makespan_s"], 1e-12)})
    if leaf == "auto":
        res["autotuner"] = leaf_for.table
        res["autotuner_leaf_sizes"] = list(leaf_for.sizes)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description="serve SPH requests on one GPU")
    ap.add_argument("--workload", choices=["evaluate", "integrate"], default="evaluate")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--budget-gib", type=float, default=None,
                    help="HBM budget (default 1 GiB for evaluate, 16 GiB for integrate)")
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--mode", choices=["native", "streams", "batched"], default="native",
                    help="native: the library's executor threads; streams: one Python "
                         "worker thread per slot; batched: one batched launch per admission")
    ap.add_argument("--load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured saturated capacity")
    ap.add_argument("--max-side", type=int, default=None)
    ap.add_argument("--block", action="store_true",
                    help="integrate on block time-steps (--steps then counts level-0 steps)")
    ap.add_argument("--leaf", default="auto",
                    help="leaf size 8, 16 or 32, or auto: the autotuner picks per request class")
    ap.add_argument("--tune-table", default=None, help="JSON table of the autotuner to load and update")
    ap.add_argument("--no-threads", action="store_true",
                    help="streams mode: drive every slot from the main thread")
    ap.add_argument("--saturated-only", action="store_true",
                    help="evaluate: serve the closed burst only (no Poisson pass)")
    ap.add_argument("--repeat", type=int, default=1,
                    help="evaluate: serve the burst this many times, 0.2 s apart")
    args = ap.parse_args(argv)
    res = run_served(args.workload, args.requests, args.steps, args.budget_gib, args.slots,
                     args.mode, args.load, args.max_side, args.leaf, args.tune_table,
                     threads=not args.no_threads, saturated_only=args.saturated_only,
                     repeat=args.repeat, block=args.block)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.exit(main())
