"""Pins of the oracle's sketched operators K_i (eq. (CT_sketches)), CPU only.

PAPER mode is the literal construction: K_l = R_l T_l for coarse levels and
K_0 = K S_r at full resolution.  UNBIASED mode replaces K_0 by
p_0^{-1}(R_0 - sum_{l>0} p_l R_l T_l) so that sum_i p_i K_i equals R_0
exactly (the constraint (si) lifted from images to operators).
"""
import numpy as np
import pytest

import oracle
import synth

G = oracle.Geometry(32, 24, 48)


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_sketch_dot_product(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.3, 0.2], mode)
    rng = np.random.default_rng(7)
    for k in range(lv.r):
        x = rng.standard_normal((32, 32))
        y = rng.standard_normal((24, 48))
        lhs = np.vdot(oracle.sketch_fwd(G, lv, k, x), y)
        rhs = np.vdot(x, oracle.sketch_adj(G, lv, k, y))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0), (k, lhs, rhs)


def test_unbiased_sketches_sum_to_full_operator():
    lv = oracle.Levels([0, 1, 2, 3], [0.25] * 4, oracle.MODE_UNBIASED)
    x = synth.random_image(32, 11)
    acc = sum(lv.p[k] * oracle.sketch_fwd(G, lv, k, x) for k in range(lv.r))
    np.testing.assert_allclose(acc, oracle.project(G, 0, x), rtol=0, atol=1e-12)
    y = synth.random_sinogram(24, 48, 12)
    acc = sum(lv.p[k] * oracle.sketch_adj(G, lv, k, y) for k in range(lv.r))
    np.testing.assert_allclose(acc, oracle.backproject(G, 0, y), rtol=0, atol=1e-12)


def test_paper_mode_on_aligned_square():
    """For x in the range of every P_l, K_0 x = R_0 x and K_l x = R_l T_l x."""
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_PAPER)
    x = synth.square_insert(32, 4, 2, 6)
    np.testing.assert_allclose(oracle.sketch_fwd(G, lv, 0, x), oracle.project(G, 0, x), atol=1e-13)
    for k in (1, 2):
        l = lv.log2f[k]
        np.testing.assert_array_equal(oracle.sketch_fwd(G, lv, k, x),
                                      oracle.project(G, l, oracle.restrict(x, l)))


def test_paper_adjoint_of_coarse_sketch():
    """K_l^T = T_l^T R_l^T = 4^{-l} T_l^* R_l^T."""
    lv = oracle.Levels([0, 2], [0.5, 0.5], oracle.MODE_PAPER)
    y = synth.random_sinogram(24, 48, 4)
    expect = oracle.prolong(oracle.backproject(G, 2, y), 2) / 16.0
    np.testing.assert_allclose(oracle.sketch_adj(G, lv, 1, y), expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_single_level_is_full_operator(mode):
    lv = oracle.Levels([0], [1.0], mode)
    x = synth.random_image(32, 1)
    np.testing.assert_allclose(oracle.sketch_fwd(G, lv, 0, x), oracle.project(G, 0, x), atol=1e-14)


def test_paper_decomposition_gap_is_small_but_nonzero():
    """Reported, not pinned to a value: R_l only approximates K T_l^*, so
    K x - sum p_i K_i x is not zero in PAPER mode (cf. the paper's Fig. 2(f))."""
    g = oracle.Geometry(64, 90, 92)
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_PAPER)
    x_true, _ = synth.ct_problem(64, 90, 92, 1e4, 1000, 2000)
    full = oracle.project(g, 0, x_true)
    acc = sum(lv.p[k] * oracle.sketch_fwd(g, lv, k, x_true) for k in range(lv.r))
    gap = np.abs(full - acc).max() / np.abs(full).max()
    assert 1e-6 < gap < 0.1
