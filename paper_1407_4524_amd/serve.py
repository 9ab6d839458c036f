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
A request the library refuses (a body that does not fit its domain) or
whose domain reports an error (LBM_E_UNSTABLE and the like) finishes as a
failed result with the error's text; its memory is released and the others
carry on.

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
    failed: bool = False
    error: str = ""

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
            batch = self.lbm.Batch(stream=stream.cuda_stream)
            # launch shapes measured on the served mix: the short rows of the
            # 3D members (46..158 nodes) are swept in spans that run across
            # rows, the 2D members in one-wavefront row tiles
            if spec["lattice"] == "D3Q19":
                batch.config = dict(batch.config, block=256, cells_per_thread=1, order=3, overlap=1)
            else:
                batch.config = dict(batch.config, block=64, cells_per_thread=1, overlap=1)
            self.groups[k] = [batch, stream]
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
        """every resident request advances n steps (enqueued on each group's
        stream); {handle: error text} of the requests whose step failed"""
        failed = {}
        by_dom = {id(dom): h for h, (_, dom) in self.handles.items()}
        for batch, _ in self.groups.values():
            if not batch.members:
                continue
            try:
                batch.step(n)
            except self.lbm.LbmError as e:
                for dom in batch.members:
                    failed[by_dom[id(dom)]] = str(e)
        return failed

    def poll(self, window, tol):
        """{handle: (steady flag, relative change, step, error text)} for every
        resident request; a request whose domain reports an error gets flag -2
        (the others of its group are checked one by one)"""
        out = {}
        by_dom = {id(dom): h for h, (_, dom) in self.handles.items()}
        for batch, _ in self.groups.values():
            if not batch.members:
                continue
            try:
                st, rel = batch.steady_state(window, tol)
            except self.lbm.LbmError:
                for dom in batch.members:
                    try:
                        s, r = dom.steady_state(window, tol) if dom.t - 1 - window >= 0 else (False, float("nan"))
                        out[by_dom[id(dom)]] = (1 if s else 0, float(r), dom.t, "")
                    except self.lbm.LbmError as e:
                        out[by_dom[id(dom)]] = (-2, float("nan"), dom.t, str(e))
                continue
            for dom, s, r in zip(batch.members, st, rel):
                out[by_dom[id(dom)]] = (int(s), float(r), dom.t, "")
        return out

    def finish(self, h):
        k, dom = self.handles.pop(h)
        ft = tuple(float(x) for x in dom.force_torque(0, dom.t - 1, 1)[0])
        self.groups[k][0].remove(dom)
        dom.close()
        return ft

    def drop(self, h):
        """releases a failed request's domain without reading its results"""
        k, dom = self.handles.pop(h)
        try:
            self.groups[k][0].remove(dom)
        except self.lbm.LbmError:
            pass
        try:
            dom.close()
        except self.lbm.LbmError:
            pass

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
                 clock=time.perf_counter, sleep=time.sleep, on_result=None):
        self.on_result = on_result  # called with every Result as it is made
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
        results = _Results(self.on_result)
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
                pending.popleft()
                try:
                    h = self.engine.start(r["spec"])
                except Exception as e:  # refused by the library: a failed result, nothing held
                    results.append(Result(r["id"], 0, False, float("nan"), (float("nan"),) * 6, r["arrival"], now,
                                          self.clock() - t0, failed=True, error=str(e)))
                    continue
                active[h] = (r, fp, now)
                used += fp
            self.peak_memory = max(self.peak_memory, used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0]["arrival"] - (self.clock() - t0)))
                continue
            step_failed = self.engine.step(self.epoch) or {}
            state = self.engine.poll(self.window, self.tol)
            done_at = self.clock() - t0
            for h in list(active):
                r, fp, adm = active[h]
                steady, rel, t, err = state[h] if len(state[h]) == 4 else (*state[h], "")
                err = step_failed.get(h, err)
                if err or steady == -2:
                    self.engine.drop(h)
                    results.append(Result(r["id"], t, False, rel, (float("nan"),) * 6, r["arrival"], adm, done_at,
                                          failed=True, error=err))
                    used -= fp
                    del active[h]
                elif steady == 1 or t >= r["max_steps"]:
                    ft = self.engine.finish(h)
                    results.append(Result(r["id"], t, steady == 1, rel, ft, r["arrival"], adm, done_at))
                    used -= fp
                    del active[h]
        return list(results)


class _Results(list):
    """A list of results that reports every one appended to a callback."""

    def __init__(self, on_result=None):
        super().__init__()
        self.on_result = on_result

    def append(self, r):
        super().append(r)
        if self.on_result:
            self.on_result(r)


def serve_plain(requests, epoch=500, window=500, tol=1e-6, record_capacity=2048, clock=time.perf_counter,
                sleep=time.sleep, on_result=None):
    """The same stream served one request at a time, each on its own domain
    and launches (lbm_step), with the same epochs and steady-state test."""
    from . import lbm
    results = _Results(on_result)
    t0 = clock()
    for r in sorted(requests, key=lambda r: r["arrival"]):
        now = clock() - t0
        if now < r["arrival"]:
            sleep(r["arrival"] - now)
        adm = clock() - t0
        try:
            dom = lbm.Domain.from_spec(r["spec"], record_capacity=record_capacity)
        except lbm.LbmError as e:  # refused by the library
            results.append(Result(r["id"], 0, False, float("nan"), (float("nan"),) * 6, r["arrival"], adm,
                                  clock() - t0, failed=True, error=str(e)))
            continue
        error = ""
        try:
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
        except lbm.LbmError as e:  # a device error (e.g. instability) fails this request only
            error, t, steady, rel, ft = str(e), dom.t, False, float("nan"), (float("nan"),) * 6
        try:
            dom.close()
        except lbm.LbmError:
            pass
        results.append(Result(r["id"], t, bool(steady), rel, ft, r["arrival"], adm, clock() - t0,
                              failed=bool(error), error=error))
    return list(results)


def summary(results, wall=None):
    """solves/s and latency percentiles of a run"""
    lat = np.array([r.latency for r in results])
    wall = wall if wall is not None else max(r.finished for r in results)
    return dict(requests=len(results), seconds=round(wall, 4), solves_per_s=round(len(results) / wall, 3),
                p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                converged=int(sum(r.converged for r in results)),
                failed=int(sum(r.failed for r in results)))
