"""Divergence guard for Alg. 1 (opt-in, host-side, off by default).

Alg. 1 contracts only for step sizes inside the admissible interval of
Sec. 3.5 (the Proposition on the step range of Thm. 3); beyond it the
parallel schedule's iterates can grow geometrically, and the first sign is
usually the dual iterate.  The guard watches a norm sampled every few
epochs and flags the run once that norm exceeds `growth` times the smallest
value seen so far, or stops being finite.  The decision is pure host logic
on the sampled norms, so it applies to the library's iterates and to the
oracle's alike.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from . import _abi


class DivergenceError(RuntimeError):
    pass


@dataclass
class Guard:
    growth: float = 1e3
    floor: float = math.inf
    history: list = field(default_factory=list)

    def update(self, epochs: float, norm: float) -> bool:
        """Record |y| after `epochs`; True when the run is judged divergent."""
        self.history.append((epochs, norm))
        if not math.isfinite(norm):
            return True
        if norm > 0.0:
            self.floor = min(self.floor, norm)
        return math.isfinite(self.floor) and norm > self.growth * self.floor


def solve_guarded(problem, budget: float, every: float = 5.0, growth: float = 1e3) -> Guard:
    """Run `budget` epochs of Alg. 1 on a Problem in chunks of `every`
    epochs, checking |y| after each; raises DivergenceError when the guard
    trips (the steps taken so far are kept)."""
    import torch

    guard = Guard(growth)
    done = 0.0
    while done < budget:
        e0 = problem.epochs
        problem.solve(min(every, budget - done), _abi.BUDGET_EPOCHS)
        done += problem.epochs - e0
        norm = float(torch.linalg.vector_norm(problem.y_cur))
        if guard.update(problem.epochs, norm):
            raise DivergenceError(f"|y| = {norm:.3e} after {problem.epochs:.1f} epochs, "
                                  f"{growth:g} x its smallest value {guard.floor:.3e}")
    return guard
