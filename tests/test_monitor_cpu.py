"""The divergence guard (paper_2412_10249_amd.monitor) on the oracle's
iterates, CPU only: on the 64^2 Tikhonov workload, Alg. 1 at Thm. 3's step
(inside the admissible interval of Sec. 3.5) runs 600 iterations without
tripping it, and at 64 times that step (far outside the interval) the dual
iterate grows geometrically and the guard trips."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import steps
from paper_2412_10249_amd.monitor import Guard

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "cfg1_sigma.json")) as f:
        return json.load(f)["paper"]


def _run(sigma, chunks=30, per=20):
    _, b = synth.ct_problem(64, 90, 92, 1e4, 1000, 2000)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    g = oracle.Geometry(64, 90, 92)
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3)
    guard = Guard(1e3)
    st = None
    for _ in range(chunks):
        st = oracle.imask_run(g, lv, oracle.Reg(lam=1e-2), sigma, 42, 0, b, per, st)
        if guard.update(st.epochs, float(np.linalg.norm(st.y))):
            return True, guard
    return False, guard


def test_guard_quiet_inside_the_admissible_interval():
    gd = _golden()
    lo, hi = steps.admissible(gd["c"], gd["rho"], gd["L2"], gd["Lbar2"], gd["Lbarp2"], 1 / 3)
    eta = gd["sigma"] / (1 + gd["sigma"])
    assert lo < eta < hi
    tripped, guard = _run(gd["sigma"])
    assert not tripped
    assert len(guard.history) == 30


def test_guard_trips_far_outside_the_admissible_interval():
    gd = _golden()
    _, hi = steps.admissible(gd["c"], gd["rho"], gd["L2"], gd["Lbar2"], gd["Lbarp2"], 1 / 3)
    sigma = 64 * gd["sigma"]
    assert sigma / (1 + sigma) > hi
    tripped, guard = _run(sigma)
    assert tripped
    norms = [n for _, n in guard.history]
    assert norms[-1] > 1e3 * min(norms)


@pytest.mark.parametrize("seq,expect", [([1.0, 2.0, 1.5, 1.9], False), ([1.0, 0.5, 600.0], True),
                                        ([0.0, 1.0, 1e4], True), ([1.0, float("nan")], True)])
def test_guard_rule(seq, expect):
    g = Guard(1e3)
    out = [g.update(float(k), v) for k, v in enumerate(seq)]
    assert out[-1] == expect and not any(out[:-1])
