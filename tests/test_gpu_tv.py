"""GPU parity of the paper's TV + nonnegativity prior (Sec. 4.5) inside
ImaSk and ImaSk-Seq against the oracle: x, y and the kept dual pair after
40 iterations within relative l2 1e-3 (FP32 against FP64 through a
nonsmooth prox), nonnegative iterates, batched = alone and resume bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu


def _run(n, na, nd, b, log2f, p, mode, lam, w, J, sigma, iters, schedule=pk.SCHEDULE_PARALLEL, theta=1.0):
    og = oracle.Geometry(n, na, nd)
    olv = oracle.Levels(list(log2f), list(p), mode)
    reg_o = oracle.Reg(oracle.REG_TV, lam=lam, tv_weight=w, tv_inner=J)
    if schedule == pk.SCHEDULE_PARALLEL:
        ost = oracle.imask_run(og, olv, reg_o, sigma, 42, 0, b, iters)
    else:
        ost = oracle.imask_seq_run(og, olv, reg_o, sigma, theta, 42, 0, b, iters)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels(tuple(log2f), tuple(p), mode),
                      pk.Regularizer(pk.REG_TV, lam, w, 0.0, J), pk.Params(sigma, 42, 0, schedule, theta), dev(b))
    prob.step(iters)
    return ost, prob


@pytest.mark.parametrize("schedule", [pk.SCHEDULE_PARALLEL, pk.SCHEDULE_SEQUENTIAL])
def test_tv_prior_parity(schedule):
    _, b = synth.ct_problem(64, 90, 92, 1e4, 1000, 2000)
    b = f32(b)
    sigma = 2e-3 if schedule == pk.SCHEDULE_PARALLEL else 1e-2
    say(f"tv prior schedule {schedule}")
    ost, prob = _run(64, 90, 92, b, (0, 1, 2, 3), (0.3, 0.3, 0.2, 0.2), pk.FULL_PAPER, 1e-2, 2e-3, 10, sigma, 40,
                     schedule)
    assert prob.epochs == ost.epochs
    x = host(prob.x_cur)
    assert x.min() >= 0.0
    assert rel(x, ost.x) <= 1e-3
    assert rel(host(prob.y_cur), ost.y) <= 1e-3
    assert rel(host(prob.tvd[prob.cur]), ost.tvd) <= 1e-3
    if schedule == pk.SCHEDULE_SEQUENTIAL:
        assert rel(host(prob.xbar), ost.xbar) <= 1e-3


def test_tv_prior_inner_counts():
    n, na, nd = 32, 30, 48
    _, b = synth.ct_problem(n, na, nd, 1e4, 1003, 2003)
    b = f32(b)
    for J in (1, 5, 12):
        ost, prob = _run(n, na, nd, b, (0, 1), (0.5, 0.5), pk.FULL_UNBIASED, 0.1, 0.05, J, 0.02, 12)
        assert rel(host(prob.x_cur), ost.x) <= 1e-3, J
        assert rel(host(prob.tvd[prob.cur]), ost.tvd) <= 1e-3, J


def test_tv_prior_batched_equals_alone_and_resume():
    geoms = [(64, 90, 92), (48, 30, 70)]
    probs, alone = [], []
    for q, (n, na, nd) in enumerate(geoms):
        _, b = synth.ct_problem(n, na, nd, 1e4, 1030 + q, 2030 + q)

        def mk():
            return pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2)),
                              pk.Regularizer(pk.REG_TV, 1e-2, 2e-3, 0.0, 8), pk.Params(2e-3, 42, q), dev(b))
        probs.append(mk())
        alone.append(mk())
    pk.step_many(probs, 16)
    for p in alone:
        p.step(8)
    saved = [p.state_dict() for p in alone]
    for p, d in zip(alone, saved):
        p.load_state_dict(d)
        p.step(8)
    torch.cuda.synchronize()
    for a, c in zip(probs, alone):
        assert torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur)
        assert torch.equal(a.tvd[a.cur], c.tvd[c.cur])


@pytest.mark.parametrize("n", [16, 64])
def test_tv_prior_prox_at_tiny_lambda_is_the_pure_prior(n):
    """With lam -> 0 the library's prox is that of the paper's prior alone
    (w TV + chi_{>=0}, Sec. 4.5): one step of one level from x^0 = v,
    y^0 = 0, zero tables and zero data has xi = 0, so x^1 is the prox at v
    with weight tau w / (1 + tau lam), tau = sigma / lam.  Against the
    oracle's dual FGP of gamma TV + chi alone (no quadratic), same J."""
    na, nd, lam, tau, w, J = 8, 14, 1e-8, 0.2, 0.5, 12
    v = synth.random_image(n, 6) * 0.5 + 0.2
    v = f32(v)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels((0,), (1.0,)),
                      pk.Regularizer(pk.REG_TV, lam, w, 0.0, J), pk.Params(tau * lam, 42, 0),
                      torch.zeros((na, nd), device="cuda"))
    prob.x[0].copy_(dev(v))
    say(f"tv prior prox at lam 1e-8, n {n}")
    prob.step(1)
    u, _ = oracle.tv_fgp(v, tau * w, J)
    x = host(prob.x_cur)
    assert x.min() >= 0.0
    assert rel(x, u) <= 1e-6, rel(x, u)
    assert np.max(np.abs(x - u)) <= 1e-6 * np.max(np.abs(u)) * 4
