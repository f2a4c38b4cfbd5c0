"""Pins of the oracle's decimation T_l, replication T_l^*, the projection
P_l = T_l^* T_l and the compensation S_r (Sec. 4.1), CPU only."""
import numpy as np
import pytest

import oracle
import synth


def test_restrict_by_hand():
    x = np.arange(16, dtype=np.float64).reshape(4, 4)
    # 2x2 block means of [[0,1,2,3],[4,5,6,7],[8,9,10,11],[12,13,14,15]]
    np.testing.assert_array_equal(oracle.restrict(x, 1), [[2.5, 4.5], [10.5, 12.5]])
    np.testing.assert_array_equal(oracle.restrict(x, 2), [[7.5]])
    np.testing.assert_array_equal(oracle.prolong(np.array([[1.0, 2.0], [3.0, 4.0]]), 1),
                                  [[1, 1, 2, 2], [1, 1, 2, 2], [3, 3, 4, 4], [3, 3, 4, 4]])


@pytest.mark.parametrize("lvl", [1, 2, 3])
def test_resampling_identities(lvl):
    n = 32
    rng = np.random.default_rng(lvl)
    x = rng.standard_normal((n, n))
    z = rng.standard_normal((n >> lvl, n >> lvl))
    # T_l T_l^* = I
    np.testing.assert_allclose(oracle.restrict(oracle.prolong(z, lvl), lvl), z, rtol=0, atol=1e-14)
    # P_l^2 = P_l, P_l symmetric
    P = lambda v: oracle.prolong(oracle.restrict(v, lvl), lvl)  # noqa: E731
    px = P(x)
    np.testing.assert_allclose(P(px), px, rtol=0, atol=1e-14)
    x2 = rng.standard_normal((n, n))
    assert abs(np.vdot(P(x), x2) - np.vdot(x, P(x2))) < 1e-12
    # the true adjoint of the block mean is 4^{-l} times replication
    assert abs(np.vdot(oracle.restrict(x, lvl), z) - np.vdot(x, oracle.prolong(z, lvl)) / 4 ** lvl) < 1e-12


def test_sketches_average_to_identity():
    """sum_i p_i S_i = I, eq. (si), with S_l = P_l for l > 0 and S_r the
    compensation (Sec. 4.1)."""
    n = 32
    lv = oracle.Levels([0, 1, 2, 3], [0.2, 0.3, 0.3, 0.2])
    x = synth.random_image(n, 5)
    acc = lv.p[0] * oracle.compensate(x, lv)
    for k in range(1, lv.r):
        acc += lv.p[k] * oracle.prolong(oracle.restrict(x, lv.log2f[k]), lv.log2f[k])
    np.testing.assert_allclose(acc, x, rtol=0, atol=1e-13)


def test_aligned_square_is_invariant():
    """The paper's square-insert image (Sec. 5) lies in every P_l's range."""
    n = 64
    x = synth.square_insert(n, 8, 2, 6)
    lv = oracle.Levels([0, 1, 2, 3], [0.25] * 4)
    for l in (1, 2, 3):
        np.testing.assert_array_equal(oracle.prolong(oracle.restrict(x, l), l), x)
    np.testing.assert_allclose(oracle.compensate(x, lv), x, rtol=0, atol=1e-14)
