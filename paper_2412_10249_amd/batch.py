"""Many independent reconstructions in flight at once.

Each problem keeps its state and workspace on the device; problems are
assigned round-robin to a few HIP streams (default priority), so the
kernels of different slices overlap on the GPU - coarse-level launches of one
slice do not fill 256 CUs by themselves.  Results are bitwise identical to
running each problem alone: the kernels are deterministic and every problem
has its own buffers.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from .imask import Problem, lib


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
