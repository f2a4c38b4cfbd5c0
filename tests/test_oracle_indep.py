"""Pins of the oracle's independent primal/dual draws (the outlook of Sec. 6),
CPU only.

  * Equal streams reproduce Alg. 1 exactly (the same draws on both sides).
  * With independent streams the two index sequences differ, each follows
    the published SplitMix64 stream of its id, and the epoch count is the
    mean of the two sides' level costs.
  * Tikhonov: the iterates converge to the dense minimiser of
    1/2|Kbar x - b|^2 + lam/2 |x|^2 (UNBIASED sketches, so Kbar = R_0).
  * Fixed point: the saddle point with consistent tables does not move.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth

G16 = oracle.Geometry(16, 24, 24)


def test_equal_streams_reproduce_alg1():
    lv = oracle.Levels([0, 1, 2], [0.5, 0.3, 0.2])
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1018, 2018)
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=0.1, tv_weight=0.02, tv_eps=0.05, tv_inner=4)
    a = oracle.imask_run(G16, lv, reg, 0.02, 42, 5, b, 30)
    c = oracle.imask_indep_run(G16, lv, reg, 0.02, 42, 5, 5, b, 30)
    assert np.array_equal(a.x, c.x) and np.array_equal(a.y, c.y)
    assert np.array_equal(a.phi, c.phi) and np.array_equal(a.psi, c.psi)
    assert a.draws == c.draws == c.dual_draws and a.epochs == c.epochs


def test_independent_streams_draws_and_epochs():
    lv = oracle.Levels([0, 1, 3], [0.3, 0.3, 0.4], oracle.MODE_UNBIASED)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1019, 2019)
    st = oracle.imask_indep_run(G16, lv, oracle.Reg(lam=0.5), 0.02, 42, 0, 1, b, 40)
    assert st.draws == list(oracle.draws(42, 0, 0, 40, lv.p))
    assert st.dual_draws == list(oracle.draws(42, 1, 0, 40, lv.p))
    assert st.draws != st.dual_draws
    cost = [1 + 0.5 + 0.125, 0.5, 0.125]
    assert abs(st.epochs - sum(0.5 * (cost[i] + cost[j]) for i, j in zip(st.draws, st.dual_draws))) < 1e-12


def test_independent_draws_converge_to_minimiser():
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_UNBIASED)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1020, 2020)
    K = oracle.dense_matrix(lambda e: oracle.project(G16, 0, e), (16, 16), 576)
    lam = 1.0
    xs = sl.cho_solve(sl.cho_factor(K.T @ K + lam * np.eye(256)), K.T @ b.ravel())
    st = None
    errs = []
    for _ in range(25):
        st = oracle.imask_indep_run(G16, lv, oracle.Reg(lam=lam), 0.01, 42, 0, 7, b, 100, st)
        errs.append(np.linalg.norm(st.x.ravel() - xs) / np.linalg.norm(xs))
    assert errs[-1] < 1e-10 and errs[-1] < 1e-6 * errs[0]


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_independent_draws_fixed_point(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.25, 0.25], mode)
    Ks = [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(G16, lv, k, e), (16, 16), 576) for k in range(3)]
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1021, 2021)
    lam = 0.1
    xs = sl.cho_solve(sl.cho_factor(Kb.T @ Kb + lam * np.eye(256)), Kb.T @ b.ravel())
    ys = Kb @ xs - b.ravel()
    st = oracle.State(xs.reshape(16, 16).copy(), ys.reshape(24, 24).copy(),
                      np.stack([(K.T @ ys).reshape(16, 16) for K in Ks]),
                      np.stack([(K @ xs).reshape(24, 24) for K in Ks]))
    out = oracle.imask_indep_run(G16, lv, oracle.Reg(lam=lam), 0.05, 42, 0, 3, b, 40, st)
    np.testing.assert_allclose(out.x, st.x, rtol=0, atol=1e-11 * np.abs(xs).max())
    np.testing.assert_allclose(out.y, st.y, rtol=0, atol=1e-11 * np.abs(ys).max())
