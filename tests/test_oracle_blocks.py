"""Pins of the oracle's image sketches combined with measurement blocks (the
outlook of Sec. 6: measurement sub-selection with image sketches), CPU only.
Alg. 1 runs over the product family K_ij = S E_j K_i (S contiguous angle
blocks, block j uniform, E_j keeping block j's rows).

  * S = 1 is Alg. 1, bit for bit.
  * The blocks partition the angles; block draws are uniform, follow the low
    word of the same SplitMix64 output as the sketch draw and are
    independent of it (joint chi-square).
  * The family averages to the level sketches: sum_ij p_i q_j K_ij = Kbar,
    tested through dense matrices built column by column.
  * Tikhonov: the iterates converge to the dense minimiser of
    1/2|Kbar x - b|^2 + lam/2 |x|^2 (UNBIASED, so Kbar = R_0).
  * Fixed point: the saddle point with consistent tables does not move.
  * Epochs: each step costs its level's cost times its block's row share.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth

G16 = oracle.Geometry(16, 24, 24)


def test_one_block_is_alg1():
    lv = oracle.Levels([0, 1, 2], [0.5, 0.3, 0.2])
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1030, 2030)
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=0.1, tv_weight=0.02, tv_eps=0.05, tv_inner=4)
    a = oracle.imask_run(G16, lv, reg, 0.02, 42, 5, b, 30)
    c = oracle.imask_blocks_run(G16, lv, reg, 0.02, 42, 5, 1, b, 30)
    assert np.array_equal(a.x, c.x) and np.array_equal(a.y, c.y)
    assert np.array_equal(a.phi, c.phi) and np.array_equal(a.psi, c.psi)
    assert a.draws == c.draws and c.blocks == [0] * 30 and a.epochs == c.epochs


def test_blocks_partition_and_draws():
    for na, S in ((24, 4), (25, 4), (7, 7), (90, 8)):
        rows = [oracle.block_rows(na, S, j) for j in range(S)]
        assert rows[0][0] == 0 and rows[-1][1] == na
        assert all(rows[j][1] == rows[j + 1][0] and rows[j][1] > rows[j][0] for j in range(S - 1))
    # the low word of SplitMix64 output k of the stream, scaled to S
    ss = oracle.splitmix64(42, 3)
    expect = [((oracle.splitmix64(ss, k) & 0xffffffff) * 5) >> 32 for k in range(200)]
    assert oracle.block_draws(42, 3, 0, 200, 5) == expect
    # joint frequencies of (level, block) against p_i / S
    p = [0.5, 0.3, 0.2]
    n = 60000
    i = oracle.draws(7, 0, 0, n, p)
    j = oracle.block_draws(7, 0, 0, n, 4)
    counts = np.zeros((3, 4))
    np.add.at(counts, (np.asarray(i), np.asarray(j)), 1)
    expected = n * np.outer(p, [0.25] * 4)
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 32.9  # 11 degrees of freedom, p = 0.0005


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_family_averages_to_the_level_sketches(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.3, 0.2], mode)
    S = 3
    Ks = [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(G16, lv, k, e), (16, 16), 576) for k in range(3)]
    Kbar = sum(p * K for p, K in zip(lv.p, Ks))
    total = np.zeros_like(Kbar)
    for k in range(3):
        for j in range(S):
            a0, a1 = oracle.block_rows(24, S, j)
            Ekj = np.zeros_like(Ks[k])
            Ekj[a0 * 24:a1 * 24] = S * Ks[k][a0 * 24:a1 * 24]
            total += lv.p[k] / S * Ekj
    np.testing.assert_allclose(total, Kbar, rtol=0, atol=1e-13 * np.abs(Kbar).max())
    if mode == oracle.MODE_UNBIASED:
        R0 = oracle.dense_matrix(lambda e: oracle.project(G16, 0, e), (16, 16), 576)
        np.testing.assert_allclose(Kbar, R0, rtol=0, atol=1e-12 * np.abs(R0).max())


def test_blocks_converge_to_minimiser():
    lv = oracle.Levels([0, 1], [0.5, 0.5], oracle.MODE_UNBIASED)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1031, 2031)
    K = oracle.dense_matrix(lambda e: oracle.project(G16, 0, e), (16, 16), 576)
    lam = 1.0
    xs = sl.cho_solve(sl.cho_factor(K.T @ K + lam * np.eye(256)), K.T @ b.ravel())
    st = None
    errs = []
    for _ in range(40):
        st = oracle.imask_blocks_run(G16, lv, oracle.Reg(lam=lam), 0.004, 42, 0, 3, b, 150, st)
        errs.append(np.linalg.norm(st.x.ravel() - xs) / np.linalg.norm(xs))
    assert errs[-1] < 1e-9 and errs[-1] < 1e-8 * errs[0], errs[::5]
    # linear rate: the error falls steadily, chunk over chunk
    assert all(b2 < 0.8 * b1 for b1, b2 in zip(errs[::5], errs[5::5]))


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_blocks_fixed_point(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.25, 0.25], mode)
    S = 4
    Ks = [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(G16, lv, k, e), (16, 16), 576) for k in range(3)]
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1032, 2032)
    lam = 0.1
    xs = sl.cho_solve(sl.cho_factor(Kb.T @ Kb + lam * np.eye(256)), Kb.T @ b.ravel())
    ys = Kb @ xs - b.ravel()
    phi = np.zeros((3 * S, 16, 16))
    psi = np.stack([(K @ xs).reshape(24, 24) for K in Ks]) * S  # K_ij x on block j's rows
    for k in range(3):
        for j in range(S):
            a0, a1 = oracle.block_rows(24, S, j)
            yj = np.zeros(576)
            yj[a0 * 24:a1 * 24] = ys[a0 * 24:a1 * 24]
            phi[k * S + j] = (S * Ks[k].T @ yj).reshape(16, 16)
    st = oracle.BlocksState(xs.reshape(16, 16).copy(), ys.reshape(24, 24).copy(), phi, psi)
    out = oracle.imask_blocks_run(G16, lv, oracle.Reg(lam=lam), 0.05, 42, 0, S, b, 40, st)
    np.testing.assert_allclose(out.x, st.x, rtol=0, atol=1e-11 * np.abs(xs).max())
    np.testing.assert_allclose(out.y, st.y, rtol=0, atol=1e-11 * np.abs(ys).max())


def test_block_epochs():
    lv = oracle.Levels([0, 1, 3], [0.3, 0.3, 0.4], oracle.MODE_UNBIASED)
    _, b = synth.ct_problem(16, 25, 24, 1e4, 1033, 2033)
    g = oracle.Geometry(16, 25, 24)
    st = oracle.imask_blocks_run(g, lv, oracle.Reg(lam=0.5), 0.02, 42, 0, 4, b, 40)
    cost = [1 + 0.5 + 0.125, 0.5, 0.125]
    share = [(lambda r: (r[1] - r[0]) / 25)(oracle.block_rows(25, 4, j)) for j in range(4)]
    assert abs(st.epochs - sum(cost[i] * share[j] for i, j in zip(st.draws, st.blocks))) < 1e-12
    assert st.draws == list(oracle.draws(42, 0, 0, 40, lv.p))
