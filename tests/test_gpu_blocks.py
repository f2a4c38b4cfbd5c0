"""GPU parity of image sketches combined with measurement blocks (the
outlook of Sec. 6, read as Alg. 1 over K_kb = S E_b K_k) against the FP64
oracle: the block draws bitwise, the epochs exactly, x, y and every table
within 1e-4 after 40 iterations (smoothed TV 1e-3); one block is Alg. 1 bit
for bit; batched = alone and resume bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu


def _data(n, na, nd, seed):
    _, b = synth.ct_problem(n, na, nd, 1e4, 1000 + seed, 2000 + seed)
    return f32(b)


def _run_both(n, na, nd, b, log2f, p, mode, S, reg_o, reg_g, sigma, iters):
    og = oracle.Geometry(n, na, nd)
    ost = oracle.imask_blocks_run(og, oracle.Levels(list(log2f), list(p), mode), reg_o, sigma, 42, 0, S, b, iters)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels(tuple(log2f), tuple(p), mode, S), reg_g,
                      pk.Params(sigma, 42, 0), dev(b))
    prob.step(iters)
    return ost, prob


def test_block_draws_match_oracle():
    lv = pk.Levels((0, 1, 2), (0.5, 0.3, 0.2), pk.FULL_PAPER, 5)
    prm = pk.Params(0.01, 42, 3)
    assert list(pk.block_draws(prm, lv, 7, 500)) == oracle.block_draws(42, 3, 7, 500, 5)
    assert list(pk.draws(prm, lv, 7, 500)) == list(oracle.draws(42, 3, 7, 500, lv.p))
    assert not pk.block_draws(prm, pk.Levels((0, 1, 2), (0.5, 0.3, 0.2)), 0, 50).any()


@pytest.mark.parametrize("mode", [pk.FULL_PAPER, pk.FULL_UNBIASED])
def test_blocks_tikhonov_parity(mode):
    n, na, nd, S = 64, 90, 92, 4
    b = _data(n, na, nd, 0)
    log2f, p = (0, 1, 2), (0.4, 0.3, 0.3)
    say(f"blocks S={S} mode {mode}")
    ost, prob = _run_both(n, na, nd, b, log2f, p, mode, S, oracle.Reg(lam=1e-2),
                          pk.Regularizer(pk.REG_TIKHONOV, 1e-2), 0.01, 40)
    assert prob.k == ost.k == 40
    assert prob.epochs == pytest.approx(ost.epochs, rel=1e-12, abs=1e-12)
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
    assert rel(host(prob.psi), ost.psi) <= 1e-4
    for j in range(S):
        for k, (l, ph) in enumerate(zip(log2f, prob.phi_tables(j))):
            exp = ost.phi[k * S + j]
            got = oracle.prolong(host(ph), l)
            assert np.linalg.norm(got - exp) <= 1e-4 * max(np.linalg.norm(exp), 1e-12) + 1e-12, (j, k)


def test_blocks_single_level_and_ragged_blocks():
    """One level (SAGA over angle blocks), 7 blocks of 90 angles (sizes 12 and 13)."""
    n, na, nd, S = 48, 90, 70, 7
    b = _data(n, na, nd, 1)
    ost, prob = _run_both(n, na, nd, b, (0,), (1.0,), pk.FULL_PAPER, S, oracle.Reg(lam=0.5),
                          pk.Regularizer(pk.REG_TIKHONOV, 0.5), 0.03, 40)
    assert prob.epochs == pytest.approx(ost.epochs, rel=1e-12)
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4


def test_blocks_smooth_tv_parity():
    n, na, nd, S = 64, 90, 92, 3
    b = _data(n, na, nd, 0)
    reg_o = oracle.Reg(oracle.REG_SMOOTH_TV, lam=1e-2, tv_weight=2e-3, tv_eps=1e-2, tv_inner=10)
    reg_g = pk.Regularizer(pk.REG_SMOOTH_TV, 1e-2, 2e-3, 1e-2, 10)
    ost, prob = _run_both(n, na, nd, b, (0, 1, 2, 3), (0.25,) * 4, pk.FULL_PAPER, S, reg_o, reg_g, 2e-3, 40)
    assert rel(host(prob.x_cur), ost.x) <= 1e-3
    assert rel(host(prob.y_cur), ost.y) <= 1e-3


def test_one_block_is_alg1_bitwise():
    n, na, nd = 64, 90, 92
    b = dev(_data(n, na, nd, 0))
    mk = lambda nb: pk.Problem(pk.Geometry(n, na, nd), pk.Levels((0, 1, 2), (0.4, 0.3, 0.3), pk.FULL_PAPER, nb),  # noqa: E731
                               pk.Regularizer(pk.REG_TIKHONOV, 1e-2), pk.Params(0.01, 42, 0), b)
    a, c = mk(0), mk(1)
    a.step(25)
    c.step(25)
    assert np.array_equal(host(a.x_cur), host(c.x_cur)) and np.array_equal(host(a.y_cur), host(c.y_cur))
    assert a.epochs == c.epochs


def test_blocks_batched_equals_alone_and_resume():
    n, na, nd = 64, 90, 92
    lv = pk.Levels((0, 1, 2), (0.4, 0.3, 0.3), pk.FULL_UNBIASED, 5)
    mk = lambda s: pk.Problem(pk.Geometry(n, na, nd), lv, pk.Regularizer(pk.REG_TIKHONOV, 1e-2),  # noqa: E731
                              pk.Params(0.01, 42, s), dev(_data(n, na, nd, s)))
    alone = [mk(s) for s in range(3)]
    for p in alone:
        p.step(20)
    batch = [mk(s) for s in range(3)]
    pk.step_many(batch, 20)
    for a, c in zip(alone, batch):
        assert np.array_equal(host(a.x_cur), host(c.x_cur)) and np.array_equal(host(a.phi), host(c.phi))
    full = mk(0)
    full.step(20)
    half = mk(0)
    half.step(8)
    snap = half.state_dict()
    other = mk(0)
    other.load_state_dict(snap)
    other.step(12)
    assert np.array_equal(host(full.x_cur), host(other.x_cur)) and np.array_equal(host(full.y_cur), host(other.y_cur))
