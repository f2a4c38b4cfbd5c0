"""Many independent reconstructions in flight at once.

Two ways to run them:
* `Batch` uses the library's batched steps: every kernel variant of a step
  is one persistent launch over the work items of all problems, the sketch
  draws happen on the device, and one captured step (a CUDA graph) is
  replayed for every step;
* `BatchGroups` splits the problems into a few such batches (sizes dealt
  round-robin, largest first) and replays each batch's captured step on a
  stream of its own, so the batches' phases overlap;
* `BatchRunner` deals the problems round-robin to a few HIP streams
  (default priority), so one slice's launches overlap another's.

Either way each problem's result is bitwise that of the problem run alone:
the kernels are deterministic and every problem has its own buffers.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from .imask import ImaskError, Problem, _stream, check, lib


def footprint_bytes(p: Problem) -> int:
    """Device bytes one problem holds (state tables + workspace)."""
    ts = [*p.x, *p.y, p.phi, p.psi, p.work, p.b, *p.tvd]
    ts += [t for t in (p.xbar, p.ztab) if t is not None]
    return sum(t.numel() * t.element_size() for t in ts)


def state_bytes(geom, levels, compact_tables: bool = False) -> int:
    """Bytes a problem of this geometry and level set will need, before
    allocating it (parallel schedule, Tikhonov or smoothed TV).  Compact
    dual tables (Remark 1) keep m + sum d_l floats instead of r m."""
    g = geom.c()
    work = lib().imask_workspace_bytes(ctypes.byref(g))
    nphi = lib().imask_phi_floats(ctypes.byref(g), ctypes.byref(levels.c()))
    m = geom.n_angles * geom.n_det
    d = geom.n * geom.n
    dual_tables = m + nphi if compact_tables else levels.r * m
    return int(work + 4 * (2 * d + 2 * m + nphi + dual_tables + m))


class BatchRunner:
    """Advances a list of Problems concurrently on `n_streams` streams."""

    def __init__(self, problems: list, n_streams: int = 8):
        self.problems = problems
        self.streams = [torch.cuda.Stream() for _ in range(max(1, n_streams))]
        producer = torch.cuda.current_stream()
        for s in self.streams:  # state was zero-filled on the current stream
            s.wait_stream(producer)

    def stream_of(self, i: int) -> torch.cuda.Stream:
        return self.streams[i % len(self.streams)]

    def step_all(self, n_steps: int = 1) -> None:
        for i, p in enumerate(self.problems):
            with torch.cuda.stream(self.stream_of(i)):
                p.step(n_steps)

    def solve_all(self, budget: float, kind: int = _abi.BUDGET_EPOCHS) -> None:
        for i, p in enumerate(self.problems):
            with torch.cuda.stream(self.stream_of(i)):
                p.solve(budget, kind)

    def synchronize(self) -> None:
        for s in self.streams:
            s.synchronize()
        torch.cuda.current_stream().wait_stream(self.streams[0])


class Batch:
    """Problems of mixed sizes advanced together by imask_batch_step until
    each has run `budget` more epochs (or iterations)."""

    def __init__(self, problems: list, budget: float, kind: int = _abi.BUDGET_EPOCHS):
        n = len(problems)
        if n == 0:
            raise ImaskError("empty batch")
        self.problems = problems
        self.n = n
        self.G = (_abi.Geometry * n)(*[p.geom.c() for p in problems])
        self.L = (_abi.Levels * n)(*[p.levels.c() for p in problems])
        self.R = (_abi.Reg * n)(*[p.reg.c() for p in problems])
        self.P = (_abi.Params * n)(*[p.params.c() for p in problems])
        self.B = (ctypes.c_void_p * n)(*[p.b.data_ptr() for p in problems])
        self.S = (_abi.State * n)(*[p._cstate() for p in problems])
        nbytes = lib().imask_batch_bytes(n, self.G, self.L)
        if nbytes == 0:
            raise ImaskError("imask_batch_bytes: invalid problems")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=problems[0].b.device)
        steps = ctypes.c_int64()
        check(lib().imask_batch_prepare(n, self.G, self.L, self.R, self.P, self.B, self.S, float(budget), kind,
                                        self.buf.data_ptr(), nbytes, ctypes.byref(steps), _stream()),
              "imask_batch_prepare")
        self.steps = int(steps.value)
        self.graph = None

    def step(self, n_steps: int = 1) -> None:
        """Enqueue n_steps batched steps on the current stream."""
        check(lib().imask_batch_step(self.n, self.G, self.L, self.buf.data_ptr(), n_steps, _stream()),
              "imask_batch_step")

    def step_overlapped(self) -> None:
        """One batched step with its forward half on the current stream and
        its transpose half on a side stream (fork after the plan, join
        before the advance)."""
        main = torch.cuda.current_stream()
        if getattr(self, "side", None) is None:
            self.side = torch.cuda.Stream()
        args = (self.n, self.G, self.L, self.buf.data_ptr())

        def part(which):
            check(lib().imask_batch_step_part(*args, which, _stream()), "imask_batch_step_part")

        part(_abi.BATCH_PLAN)
        fork = torch.cuda.Event()
        fork.record(main)
        self.side.wait_event(fork)
        part(_abi.BATCH_FORWARD)
        with torch.cuda.stream(self.side):
            part(_abi.BATCH_TRANSPOSE)
        join = torch.cuda.Event()
        join.record(self.side)
        main.wait_event(join)
        part(_abi.BATCH_ADVANCE)

    def capture(self, overlapped: bool = False) -> None:
        """Record one batched step in a CUDA graph (nothing runs yet);
        `overlapped` puts its two halves on two streams."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            if overlapped:
                self.step_overlapped()
            else:
                self.step(1)
        self.graph = g

    def replay(self, n_steps: int = 1) -> None:
        for _ in range(n_steps):
            self.graph.replay()

    def run(self, graph: bool = True) -> None:
        """All the steps the budgets need, from a replayed graph or eagerly."""
        if graph:
            if self.graph is None:
                self.capture()
            self.replay(self.steps)
        else:
            self.step(self.steps)

    def sync_state(self) -> None:
        """Copy the device counters back into the Problems (synchronises)."""
        check(lib().imask_batch_state(self.n, self.L, self.buf.data_ptr(), self.S, _stream()), "imask_batch_state")
        for p, s in zip(self.problems, self.S):
            p._absorb(s)


class BatchGroups:
    """The problems in `groups` batches, one HIP stream each (default
    priority): every batch's step is captured once and replayed on its
    stream, so one batch's transposes overlap another's forward passes.  A
    box exposes few hardware queues (four here), about as many groups as
    pay off."""

    def __init__(self, problems, budget: float, kind: int = _abi.BUDGET_ITERS, groups: int = 4):
        order = sorted(range(len(problems)), key=lambda q: -problems[q].geom.n)
        self.groups = [Batch([problems[q] for q in order[g::groups]], budget, kind)
                       for g in range(min(groups, len(problems)))]
        self.streams = [torch.cuda.Stream() for _ in self.groups]

    def capture(self) -> None:
        for bt, st in zip(self.groups, self.streams):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                bt.capture()

    def run(self) -> None:
        """Every batch's steps on its stream; the current stream waits for all."""
        if any(bt.graph is None for bt in self.groups):
            self.capture()
        main = torch.cuda.current_stream()
        for bt, st in zip(self.groups, self.streams):
            st.wait_stream(main)
            with torch.cuda.stream(st):
                bt.replay(bt.steps)
        for st in self.streams:
            main.wait_stream(st)

    def sync_state(self) -> None:
        for bt in self.groups:
            bt.sync_state()
