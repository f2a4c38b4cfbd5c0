"""Pins of the oracle's compact dual tables (Remark 1: keep the iterate
instead of its projection, and a running table average), CPU only.

In exact arithmetic the compact variant is Alg. 1 itself: one projection of
the difference x^k - z_i gives psi_new - psi_i.  So, over many iterations,
its iterates equal the standard oracle's to FP64 rounding, and its table
average equals sum_i p_i psi_i of the standard run.  Both sketch modes and
both regularisers are covered.
"""
import numpy as np
import pytest

import oracle
import synth

G16 = oracle.Geometry(16, 24, 24)


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
@pytest.mark.parametrize("kind", [oracle.REG_TIKHONOV, oracle.REG_TV])
def test_compact_tables_equal_alg1(mode, kind):
    lv = oracle.Levels([0, 1, 2], [0.4, 0.35, 0.25], mode)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1016, 2016)
    reg = oracle.Reg(kind, lam=0.5, tv_weight=0.02, tv_inner=6)
    std = oracle.imask_run(G16, lv, reg, 0.02, 42, 3, b, 120)
    cmp_ = oracle.imask_compact_run(G16, lv, reg, 0.02, 42, 3, b, 120)
    assert std.draws == cmp_.draws and std.epochs == cmp_.epochs
    for a, c in ((std.x, cmp_.x), (std.y, cmp_.y), (std.phi, cmp_.phi)):
        assert np.linalg.norm(a - c) <= 1e-12 * np.linalg.norm(a)
    psibar = sum(pk * std.psi[k] for k, pk in enumerate(lv.p))
    assert np.linalg.norm(psibar - cmp_.psibar) <= 1e-12 * np.linalg.norm(psibar)


def test_compact_resume_is_bitwise():
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1017, 2017)
    reg = oracle.Reg(lam=0.3)
    whole = oracle.imask_compact_run(G16, lv, reg, 0.02, 42, 1, b, 30)
    half = oracle.imask_compact_run(G16, lv, reg, 0.02, 42, 1, b, 15)
    rest = oracle.imask_compact_run(G16, lv, reg, 0.02, 42, 1, b, 15, half)
    for a, c in ((whole.x, rest.x), (whole.y, rest.y), (whole.z, rest.z), (whole.psibar, rest.psibar)):
        assert np.array_equal(a, c)
