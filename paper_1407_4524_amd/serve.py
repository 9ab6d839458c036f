"""Serving loop: drag/torque solve requests of different sizes, admitted as
device memory and batch slots free up (continuous batching).

Requests arrive over time. The scheduler admits them in arrival order while
the sum of their device footprints (``lbm_footprint_bytes`` +
``lbm_body_footprint_bytes``) stays within the memory budget and the number
of resident requests within ``max_active``; an admitted request's
populations, link list and records stay resident on the device until it
finishes. Every epoch each resident request advances ``epoch`` steps --
requests of one lattice, storage and equilibrium share a batch (one set of
launches per step), batches run on streams of their own so their work
overlaps on the device -- and then the FP64 steady-state check runs on the
device for all of them at once. A request finishes when its drag changes by
less than ``tol`` (relative) over ``window`` steps, or at ``max_steps``
(checked at epoch boundaries); it then leaves, and its memory admits the
next waiting request at once. The batched arithmetic is that of a domain
stepped alone, so a result does not depend on the mix it was served in.

``serve_plain`` serves the same stream one request at a time with one
domain per launch, the reference the batched loop is measured against.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Result:
    id: int
    steps: int
    converged: bool
    rel_change: float
    force_torque: tuple  # (Fx, Fy, Fz, Tx, Ty, Tz) at the last step
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self):
        return self.finished - self.arrival


class GpuEngine:
    """Resident requests on the GPU: one batch and one stream per (lattice,
    storage, equilibrium) group."""

    def __init__(self, record_capacity=2048):
        import torch
        from . import lbm
        self.torch = torch
        self.lbm = lbm
        self.record_capacity = record_capacity
        self.groups = {}  # key -> [Batch, torch stream]
        self.handles = {}  # handle -> (key, Domain)
        self._next = 0

    @staticmethod
    def key(spec):
        return (spec["lattice"], spec["storage"], spec.get("eq", "bgk"))

    def footprint(self, spec):
        return self.lbm.footprint_bytes(spec, record_capacity=self.record_capacity)

    def start(self, spec):
        k = self.key(spec)
        if k not in self.groups:
            stream = self.torch.cuda.Stream()  # default priority
            self.groups[k] = [self.lbm.Batch(stream=stream.cuda_stream), stream]
        batch, stream = self.groups[k]
        with self.torch.cuda.stream(stream):
            dom = self.lbm.Domain.from_spec(spec, record_capacity=self.record_capacity,
                                            stream=stream.cuda_stream)
        batch.add(dom)
        h = self._next
        self._next += 1
        self.handles[h] = (k, dom)
        return h

    def step(self, n):
        """every resident request advances n steps (enqueued on each group's stream)"""
        for batch, _ in self.groups.values():
            if batch.members:
                batch.step(n)

    def poll(self, window, tol):
        """{handle: (steady flag, relative change, step)} for every resident request"""
        out = {}
        by_dom = {id(dom): h for h, (_, dom) in self.handles.items()}
        for batch, _ in self.groups.values():
            if not batch.members:
                continue
            st, rel = batch.steady_state(window, tol)
            for dom, s, r in zip(batch.members, st, rel):
                out[by_dom[id(dom)]] = (int(s), float(r), dom.t)
        return out

    def finish(self, h):
        k, dom = self.handles.pop(h)
        ft = tuple(float(x) for x in dom.force_torque(0, dom.t - 1, 1)[0])
        self.groups[k][0].remove(dom)
        dom.close()
        return ft

    def close(self):
        for h in list(self.handles):
            self.finish(h)
        for batch, _ in self.groups.values():
            batch.close()
        self.groups = {}


class Server:
    """Continuous-batching scheduler over an engine (see the module text).
    The engine is anything with footprint/start/step/poll/finish, so the
    scheduling logic runs without a GPU in the tests."""

    def __init__(self, engine, memory_budget, max_active=256, epoch=500, window=500, tol=1e-6,
                 clock=time.perf_counter, sleep=time.sleep):
        self.engine = engine
        self.budget = int(memory_budget)
        self.max_active = max_active
        self.epoch = epoch
        self.window = window
        self.tol = tol
        self.clock = clock
        self.sleep = sleep
        self.peak_memory = 0
        self.peak_active = 0
        self.rejected = []

    def run(self, requests):
        """Serves the requests (dictionaries with id, arrival [s], spec,
        max_steps) and returns their Results in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        active = {}  # handle -> (request, footprint, admitted)
        used = 0
        results = []
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            while pending and pending[0]["arrival"] <= now:
                r = pending[0]
                fp = self.engine.footprint(r["spec"])
                if fp > self.budget:
                    self.rejected.append(r["id"])
                    pending.popleft()
                    continue
                if used + fp > self.budget or len(active) >= self.max_active:
                    break  # the head waits; no later request overtakes it
                h = self.engine.start(r["spec"])
                active[h] = (r, fp, now)
                used += fp
                pending.popleft()
            self.peak_memory = max(self.peak_memory, used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0]["arrival"] - (self.clock() - t0)))
                continue
            self.engine.step(self.epoch)
            state = self.engine.poll(self.window, self.tol)
            done_at = self.clock() - t0
            for h in list(active):
                r, fp, adm = active[h]
                steady, rel, t = state[h]
                if steady == 1 or t >= r["max_steps"]:
                    ft = self.engine.finish(h)
                    results.append(Result(r["id"], t, steady == 1, rel, ft, r["arrival"], adm, done_at))
                    used -= fp
                    del active[h]
        return results


def serve_plain(requests, epoch=500, window=500, tol=1e-6, record_capacity=2048, clock=time.perf_counter,
                sleep=time.sleep):
    """The same stream served one request at a time, each on its own domain
    and launches (lbm_step), with the same epochs and steady-state test."""
    from . import lbm
    results = []
    t0 = clock()
    for r in sorted(requests, key=lambda r: r["arrival"]):
        now = clock() - t0
        if now < r["arrival"]:
            sleep(r["arrival"] - now)
        adm = clock() - t0
        dom = lbm.Domain.from_spec(r["spec"], record_capacity=record_capacity)
        while True:
            dom.step(epoch)
            t = dom.t
            if t - 1 - window >= 0:
                steady, rel = dom.steady_state(window, tol)
            else:
                steady, rel = False, float("nan")
            if steady or t >= r["max_steps"]:
                break
        ft = tuple(float(x) for x in dom.force_torque(0, t - 1, 1)[0])
        dom.close()
        results.append(Result(r["id"], t, bool(steady), rel, ft, r["arrival"], adm, clock() - t0))
    return results


def summary(results, wall=None):
    """solves/s and latency percentiles of a run"""
    lat = np.array([r.latency for r in results])
    wall = wall if wall is not None else max(r.finished for r in results)
    return dict(requests=len(results), seconds=round(wall, 4), solves_per_s=round(len(results) / wall, 3),
                p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                converged=int(sum(r.converged for r in results)))
