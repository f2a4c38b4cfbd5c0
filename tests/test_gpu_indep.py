"""GPU parity of independent primal/dual sketch draws (Sec. 6 outlook)
against the oracle: both index streams and the epoch count exact, x and y
after 50 iterations within relative l2 1e-4 (smoothed TV 1e-3); with equal
streams the run is bitwise the common-draw run.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu

IND = pk.DRAW_INDEPENDENT


@pytest.mark.parametrize("mode", [pk.FULL_PAPER, pk.FULL_UNBIASED])
def test_independent_draws_parity(mode):
    n, na, nd = 64, 90, 92
    _, b = synth.ct_problem(n, na, nd, 1e4, 1000, 2000)
    b = f32(b)
    log2f, p = (0, 1, 2, 3), (0.3, 0.3, 0.2, 0.2)
    say(f"independent draws mode {mode}")
    ost = oracle.imask_indep_run(oracle.Geometry(n, na, nd), oracle.Levels(list(log2f), list(p), mode),
                                 oracle.Reg(lam=0.5), 0.02, 42, 0, 9, b, 50)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels(log2f, p, mode), pk.Regularizer(pk.REG_TIKHONOV, 0.5),
                      pk.Params(0.02, 42, 0, draw_mode=IND, dual_stream_id=9), dev(b))
    prob.step(50)
    assert prob.epochs == ost.epochs
    assert list(pk.draws(pk.Params(0.02, 42, 0), prob.levels, 0, 50)) == ost.draws
    assert list(pk.draws(pk.Params(0.02, 42, 9), prob.levels, 0, 50)) == ost.dual_draws
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
    assert rel(host(prob.psi), ost.psi) <= 1e-4


def test_independent_draws_smooth_tv():
    n, na, nd = 48, 60, 70
    _, b = synth.ct_problem(n, na, nd, 1e4, 1005, 2005)
    b = f32(b)
    reg_o = oracle.Reg(oracle.REG_SMOOTH_TV, lam=1e-2, tv_weight=2e-3, tv_eps=1e-2, tv_inner=10)
    ost = oracle.imask_indep_run(oracle.Geometry(n, na, nd), oracle.Levels([0, 1, 2], [1 / 3] * 3), reg_o, 2e-3,
                                 42, 1, 2, b, 40)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2)),
                      pk.Regularizer(pk.REG_SMOOTH_TV, 1e-2, 2e-3, 1e-2, 10),
                      pk.Params(2e-3, 42, 1, draw_mode=IND, dual_stream_id=2), dev(b))
    prob.step(40)
    assert rel(host(prob.x_cur), ost.x) <= 1e-3
    assert rel(host(prob.y_cur), ost.y) <= 1e-3


def test_equal_streams_are_common_draws_bitwise():
    n, na, nd = 64, 90, 92
    _, b = synth.ct_problem(n, na, nd, 1e4, 1006, 2006)
    geom, lv, reg = pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2)), pk.Regularizer(pk.REG_TIKHONOV, 0.1)
    a = pk.Problem(geom, lv, reg, pk.Params(0.01, 42, 4), dev(b))
    c = pk.Problem(geom, lv, reg, pk.Params(0.01, 42, 4, draw_mode=IND, dual_stream_id=4), dev(b))
    a.step(25)
    c.step(25)
    torch.cuda.synchronize()
    assert torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur) and a.epochs == c.epochs
