"""The library's batched steps (imask_batch_*) against the same problems
stepped alone with imask_step: every slice of a mixed-size batch equal bit
for bit (x, y, phi, psi, k, epochs), in PAPER and UNBIASED modes, with
iteration and epoch budgets; a captured step replayed as a CUDA graph,
each replay checked against eager batched steps of an identical batch; the
step's forward and transpose halves on two streams, eager and captured; and
the mixed 256..1024 grids of the batched workload."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, host, say

import paper_2412_10249_amd as pk
from paper_2412_10249_amd.batch import Batch, BatchGroups

pytestmark = pytest.mark.gpu


def _problems(specs, lam=1e-2, sigma=1e-3):
    out = []
    for q, (n, levels, mode) in enumerate(specs):
        na = nd = 3 * n // 2
        _, b = synth.ct_problem(n, na, nd, 1e5, 1100 + q, 2100 + q)
        out.append(pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform(levels, mode),
                              pk.Regularizer(pk.REG_TIKHONOV, lam), pk.Params(sigma, 42, 7 + q), dev(b)))
    return out


SPECS = [(64, (0, 1, 2, 3), pk.FULL_PAPER), (96, (0, 1, 2), pk.FULL_UNBIASED), (128, (0, 2), pk.FULL_PAPER),
         (48, (0, 1, 2, 3, 4), pk.FULL_UNBIASED), (32, (0,), pk.FULL_PAPER), (64, (0, 1, 2, 3), pk.FULL_UNBIASED)]


def _same(a, c):
    return (torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur) and torch.equal(a.phi, c.phi)
            and torch.equal(a.psi, c.psi) and a.k == c.k and a.epochs == c.epochs and a.cur == c.cur)


@pytest.mark.parametrize("kind,budget", [(pk.BUDGET_ITERS, 24), (pk.BUDGET_EPOCHS, 9.0)])
def test_batch_equals_alone(kind, budget):
    say(f"batch vs alone, budget {budget} kind {kind}")
    batched, alone = _problems(SPECS), _problems(SPECS)
    bt = Batch(batched, budget, kind)
    bt.run(graph=False)
    bt.sync_state()
    for p in alone:
        p.solve(budget, kind)
    torch.cuda.synchronize()
    for q, (a, c) in enumerate(zip(batched, alone)):
        assert _same(a, c), q
    assert bt.steps == max(p.k for p in alone)


def test_batch_graph_replays_equal_eager_steps():
    """One captured batched step replayed 12 times; after every replay the
    state equals that of an identical batch stepped eagerly, with
    synchronisations and eager work between the replays."""
    g_probs, e_probs = _problems(SPECS[:4]), _problems(SPECS[:4])
    gb = Batch(g_probs, 12, pk.BUDGET_ITERS)
    eb = Batch(e_probs, 12, pk.BUDGET_ITERS)
    gb.capture()
    for it in range(12):
        gb.replay(1)
        eb.step(1)
        torch.cuda.synchronize()
        _ = torch.ones(1024, device="cuda").sum().item()  # unrelated eager work between replays
        for q, (a, c) in enumerate(zip(g_probs, e_probs)):
            assert torch.equal(a.x[0], c.x[0]) and torch.equal(a.x[1], c.x[1]), (it, q)
            assert torch.equal(a.y[0], c.y[0]) and torch.equal(a.y[1], c.y[1]), (it, q)
            assert torch.equal(a.phi, c.phi) and torch.equal(a.psi, c.psi), (it, q)
    gb.sync_state()
    eb.sync_state()
    alone = _problems(SPECS[:4])
    for p in alone:
        p.step(12)
    torch.cuda.synchronize()
    for a, c in zip(g_probs, alone):
        assert _same(a, c)


@pytest.mark.parametrize("captured", [False, True])
def test_batch_two_streams_equal_one_stream(captured):
    """The step split into its parts, forward on the current stream and
    transpose on a side stream (eager, or captured once and replayed 10
    times with eager work between replays): after every step equal bit for
    bit to an identical batch stepped on one stream, and at the end to the
    problems stepped alone."""
    say(f"two-stream batched step, captured={captured}")
    o_probs, e_probs = _problems(SPECS), _problems(SPECS)
    ob = Batch(o_probs, 10, pk.BUDGET_ITERS)
    eb = Batch(e_probs, 10, pk.BUDGET_ITERS)
    if captured:
        ob.capture(overlapped=True)
    for it in range(10):
        if captured:
            ob.replay(1)
        else:
            ob.step_overlapped()
        eb.step(1)
        torch.cuda.synchronize()
        _ = torch.ones(1024, device="cuda").sum().item()
        for q, (a, c) in enumerate(zip(o_probs, e_probs)):
            assert torch.equal(a.x[0], c.x[0]) and torch.equal(a.x[1], c.x[1]), (it, q)
            assert torch.equal(a.y[0], c.y[0]) and torch.equal(a.y[1], c.y[1]), (it, q)
            assert torch.equal(a.phi, c.phi) and torch.equal(a.psi, c.psi), (it, q)
    ob.sync_state()
    alone = _problems(SPECS)
    for p in alone:
        p.step(10)
    torch.cuda.synchronize()
    for q, (a, c) in enumerate(zip(o_probs, alone)):
        assert _same(a, c), q


def test_batch_groups_equal_alone():
    """The problems split in 3 batches replayed concurrently on 3 streams:
    every problem equal bit for bit to its run alone."""
    say("batch groups")
    grouped, alone = _problems(SPECS), _problems(SPECS)
    bg = BatchGroups(grouped, 15, pk.BUDGET_ITERS, groups=3)
    bg.run()
    torch.cuda.synchronize()
    bg.sync_state()
    for p in alone:
        p.step(15)
    torch.cuda.synchronize()
    for q, (a, c) in enumerate(zip(grouped, alone)):
        assert _same(a, c), q


def test_batched_workload_grids():
    """One slice of each size of the batched workload (N = 256 ... 1024,
    angles = bins = 1.5 N, levels 0-3, PAPER), 8 iterations: equal to alone."""
    specs = [(n, (0, 1, 2, 3), pk.FULL_PAPER) for n in (256, 384, 512, 768, 1024)]
    say("batched workload grids")
    batched, alone = _problems(specs), _problems(specs)
    bt = Batch(batched, 8, pk.BUDGET_ITERS)
    bt.run(graph=True)
    bt.sync_state()
    for p in alone:
        p.step(8)
    torch.cuda.synchronize()
    for q, (a, c) in enumerate(zip(batched, alone)):
        assert _same(a, c), q
        assert np.isfinite(host(a.x_cur)).all()
