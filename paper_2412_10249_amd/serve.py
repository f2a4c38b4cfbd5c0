"""Continuous-batching reconstruction server.

Requests (a geometry and its data) arrive over time.  A request is admitted
as soon as a slot is free and its device footprint fits the HBM budget; its
iterate, dual variable and gradient tables then stay on the device until it
has done its epoch budget.  Every scheduling tick enqueues a chunk of epochs
for each active request on that request's stream, so the work of requests
admitted at different times overlaps on the GPU; a request finishes when the
event recorded after its last chunk has completed.  Latency is completion
minus arrival.

The scheduling logic (`Scheduler`) only talks to an executor interface, so
it is tested on the CPU with a simulated executor.
"""
from __future__ import annotations

import heapq
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    n: int
    arrival: float
    epochs: float
    data: object = None          # executor-specific payload (e.g. the sinogram)
    footprint: int = 0
    admitted: float | None = None
    done: float | None = None
    result: object = None

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class Executor:
    """What the scheduler needs from a device (or a simulation of one)."""

    def footprint(self, req: Request) -> int:  # bytes the request will hold
        raise NotImplementedError

    def start(self, req: Request, slot: int) -> None:
        raise NotImplementedError

    def advance(self, req: Request, epochs: float) -> None:  # enqueue, do not wait
        raise NotImplementedError

    def finished(self, req: Request) -> bool:  # epoch budget reached and the device is done
        raise NotImplementedError

    def release(self, req: Request) -> None:
        raise NotImplementedError


@dataclass
class Scheduler:
    executor: Executor
    hbm_budget: int
    max_active: int
    chunk_epochs: float = 1.0
    clock: object = time.perf_counter
    queue: list = field(default_factory=list)
    active: dict = field(default_factory=dict)  # slot -> request
    finished: list = field(default_factory=list)
    used: int = 0

    def submit(self, req: Request) -> None:
        req.footprint = self.executor.footprint(req)
        if req.footprint > self.hbm_budget:
            raise ValueError(f"request {req.rid} needs {req.footprint} bytes, budget is {self.hbm_budget}")
        self.queue.append(req)

    def _admit(self) -> None:
        # first come first served: a large head-of-line request waits for memory
        while self.queue and len(self.active) < self.max_active:
            req = self.queue[0]
            if self.used + req.footprint > self.hbm_budget:
                break
            self.queue.pop(0)
            slot = next(s for s in range(self.max_active) if s not in self.active)
            self.used += req.footprint
            req.admitted = self.clock()
            self.executor.start(req, slot)
            self.active[slot] = req

    def tick(self) -> int:
        """Admit, retire finished requests, enqueue the next chunk for the rest.
        Returns the number of active requests."""
        for slot, req in list(self.active.items()):
            if self.executor.finished(req):
                req.done = self.clock()
                self.executor.release(req)
                self.used -= req.footprint
                del self.active[slot]
                self.finished.append(req)
        self._admit()
        for req in self.active.values():
            self.executor.advance(req, self.chunk_epochs)
        return len(self.active)


def poisson_arrivals(rate: float, duration: float, seed: int = 7, sizes=(128, 256, 512, 1024),
                     weights=(4, 3, 2, 1)):
    """(time, N) pairs: exponential gaps at `rate` per second, sizes drawn with weights."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            return out
        out.append((t, int(rng.choice(sizes, p=w / w.sum()))))


def run_load(scheduler: Scheduler, arrivals, make_request, poll: float = 0.0005, drain: bool = True,
             now=time.perf_counter, sleep=time.sleep):
    """Feeds timed arrivals into the scheduler in real time (or on a
    simulated clock) and ticks until everything submitted has finished."""
    pending = list(arrivals)
    heapq.heapify(pending)
    t0 = now()
    rid = 0
    while pending or scheduler.queue or scheduler.active:
        el = now() - t0
        while pending and pending[0][0] <= el:
            ta, n = heapq.heappop(pending)
            scheduler.submit(make_request(rid, n, t0 + ta))
            rid += 1
        scheduler.tick()
        if not drain and not pending:
            break
        if not (pending or scheduler.queue or scheduler.active):
            break
        # wait one poll interval (or until the next arrival, if sooner)
        gap = pending[0][0] - (now() - t0) if pending else poll
        sleep(max(0.0, min(poll, gap)))
    return scheduler.finished


def latency_summary(reqs, t_window: float | None = None) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {"completed": 0}
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"completed": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "served_per_s": float(lat.size / span) if span > 0 else None}


class GpuExecutor(Executor):
    """Executor backed by libimask: one Problem per request, one stream per slot."""

    def __init__(self, n_slots: int, levels_for, reg, sigma_for, seed: int = 42):
        import torch

        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.levels_for, self.reg, self.sigma_for, self.seed = levels_for, reg, sigma_for, seed
        self.state = {}

    def _geom(self, req):
        from .imask import Geometry

        return Geometry(req.n, 3 * req.n // 2, 3 * req.n // 2)

    def footprint(self, req):
        from .batch import state_bytes

        return state_bytes(self._geom(req), self.levels_for(req.n))

    def start(self, req, slot):
        from .imask import Params, Problem

        torch = self.torch
        s = self.streams[slot]
        geom = self._geom(req)
        with torch.cuda.stream(s):
            b = req.data if isinstance(req.data, torch.Tensor) else torch.as_tensor(req.data, device="cuda")
            prob = Problem(geom, self.levels_for(req.n), self.reg,
                           Params(self.sigma_for(geom), self.seed, req.rid), b.float().contiguous())
        self.state[req.rid] = {"prob": prob, "stream": s, "events": []}

    def advance(self, req, epochs):
        from . import _abi

        torch = self.torch
        st = self.state[req.rid]
        prob = st["prob"]
        st["events"] = [e for e in st["events"] if not e.query()]
        left = req.epochs - prob.epochs
        if left <= 0 or len(st["events"]) >= 2:  # at most two chunks in flight per request
            return
        with torch.cuda.stream(st["stream"]):
            prob.solve(min(epochs, left), _abi.BUDGET_EPOCHS)
            ev = torch.cuda.Event()
            ev.record(st["stream"])
        st["events"].append(ev)

    def finished(self, req):
        st = self.state[req.rid]
        return st["prob"].epochs >= req.epochs and all(e.query() for e in st["events"])

    def release(self, req):
        st = self.state.pop(req.rid)
        st["stream"].synchronize()
        with self.torch.cuda.stream(st["stream"]):
            req.result = st["prob"].x_cur.clone()
        st["stream"].synchronize()
