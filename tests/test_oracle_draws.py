"""Pins of the oracle's sketch-index draw (Alg. 1: level i is picked with
probability p_i in every iteration), CPU only.

The generator is SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in counter
form; the first outputs for state 0 are the generator's published test
vector.  Index selection uses 32-bit integer thresholds of the cumulative p.
"""
import numpy as np

import oracle


def test_splitmix64_reference_outputs():
    assert oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(0, 2) == 0x06C45D188009454F


def test_thresholds():
    assert list(oracle.thresholds([0.25] * 4)) == [2 ** 30, 2 ** 31, 3 * 2 ** 30, 2 ** 32]
    assert oracle.thresholds([1.0])[0] == 2 ** 32
    t = oracle.thresholds([0.3, 0.3, 0.2, 0.2])
    assert list(t) == [int(np.floor(2 ** 32 * 0.3)), int(np.floor(2 ** 32 * 0.6)),
                       int(np.floor(2 ** 32 * (0.3 + 0.3 + 0.2))), 2 ** 32]


def test_draw_frequencies_chi_square():
    p = np.array([0.3, 0.3, 0.2, 0.2])
    n = 1_000_000
    counts = np.bincount(oracle.draws(42, 0, 0, n, p), minlength=4)
    chi2 = np.sum((counts - n * p) ** 2 / (n * p))
    assert chi2 < 16.27  # 99.9% quantile, 3 dof


def test_counter_random_access_and_streams():
    p = [1 / 3] * 3
    full = oracle.draws(42, 5, 0, 64, p)
    np.testing.assert_array_equal(oracle.draws(42, 5, 20, 44, p), full[20:])
    other = oracle.draws(42, 6, 0, 64, p)
    assert not np.array_equal(full, other)


def test_draw_rule_matches_definition():
    p = [0.5, 0.25, 0.25]
    seed, stream = 42, 3
    ss = oracle.splitmix64(seed, stream)
    d = oracle.draws(seed, stream, 0, 32, p)
    for k in range(32):
        u = oracle.splitmix64(ss, k) >> 32
        expect = 0 if u < 2 ** 31 else (1 if u < 3 * 2 ** 30 else 2)
        assert d[k] == expect
