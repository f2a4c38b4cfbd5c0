"""GPU parity of the compact dual tables (Remark 1) against the oracle's
compact variant, and against the standard tables on the GPU: x, y, phi and
the table average after 50 iterations within relative l2 1e-4; smaller
device footprint; batched = alone and resume bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk
from paper_2412_10249_amd import batch

pytestmark = pytest.mark.gpu


def _problem(geom, lv, reg, b, compact, stream=0):
    return pk.Problem(geom, lv, reg, pk.Params(0.02, 42, stream), dev(b), compact_tables=compact)


@pytest.mark.parametrize("mode", [pk.FULL_PAPER, pk.FULL_UNBIASED])
def test_compact_tables_parity(mode):
    n, na, nd = 64, 90, 92
    _, b = synth.ct_problem(n, na, nd, 1e4, 1000, 2000)
    b = f32(b)
    log2f, p = (0, 1, 2), (0.4, 0.35, 0.25)
    say(f"compact tables mode {mode}")
    ost = oracle.imask_compact_run(oracle.Geometry(n, na, nd), oracle.Levels(list(log2f), list(p), mode),
                                   oracle.Reg(lam=0.5), 0.02, 42, 0, b, 50)
    geom, lv, reg = pk.Geometry(n, na, nd), pk.Levels(log2f, p, mode), pk.Regularizer(pk.REG_TIKHONOV, 0.5)
    cp = _problem(geom, lv, reg, b, True)
    sp = _problem(geom, lv, reg, b, False)
    cp.step(50)
    sp.step(50)
    assert cp.epochs == ost.epochs
    assert rel(host(cp.x_cur), ost.x) <= 1e-4
    assert rel(host(cp.y_cur), ost.y) <= 1e-4
    assert rel(host(cp.psi), ost.psibar) <= 1e-4
    for k, (l, ph) in enumerate(zip(log2f, cp.phi_tables())):
        assert rel(oracle.prolong(host(ph), l), ost.phi[k]) <= 1e-4
    # the same iteration as the standard tables, up to FP32 rounding
    assert rel(host(cp.x_cur), host(sp.x_cur)) <= 1e-5
    avg = sum(pj * host(sp.psi[j]) for j, pj in enumerate(p))
    assert rel(host(cp.psi), avg) <= 1e-5
    assert batch.footprint_bytes(cp) < batch.footprint_bytes(sp)
    assert batch.footprint_bytes(cp) == batch.state_bytes(geom, lv, compact_tables=True)


def test_compact_tables_tv_prior():
    n, na, nd = 48, 60, 70
    _, b = synth.ct_problem(n, na, nd, 1e4, 1004, 2004)
    b = f32(b)
    ost = oracle.imask_compact_run(oracle.Geometry(n, na, nd), oracle.Levels([0, 1, 2], [1 / 3] * 3),
                                   oracle.Reg(oracle.REG_TV, lam=1e-2, tv_weight=2e-3, tv_inner=8), 2e-3, 42, 0, b, 40)
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2)), pk.Regularizer(pk.REG_TV, 1e-2, 2e-3, 0.0, 8),
                      pk.Params(2e-3, 42, 0), dev(b), compact_tables=True)
    prob.step(40)
    assert rel(host(prob.x_cur), ost.x) <= 1e-3
    assert rel(host(prob.psi), ost.psibar) <= 1e-3


def test_compact_tables_batched_and_resume():
    geoms = [(64, 90, 92), (32, 45, 50)]
    probs, alone = [], []
    for q, (n, na, nd) in enumerate(geoms):
        _, b = synth.ct_problem(n, na, nd, 1e4, 1040 + q, 2040 + q)
        mk = lambda: pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform((0, 1, 2), pk.FULL_UNBIASED),  # noqa: E731
                                pk.Regularizer(pk.REG_TIKHONOV, 0.1), pk.Params(0.01, 42, q), dev(b),
                                compact_tables=True)
        probs.append(mk())
        alone.append(mk())
    pk.step_many(probs, 20)
    for p in alone:
        p.step(10)
    saved = [p.state_dict() for p in alone]
    for p, d in zip(alone, saved):
        p.load_state_dict(d)
        p.step(10)
    torch.cuda.synchronize()
    for a, c in zip(probs, alone):
        assert torch.equal(a.x_cur, c.x_cur) and torch.equal(a.y_cur, c.y_cur)
        assert torch.equal(a.psi, c.psi) and torch.equal(a.ztab, c.ztab) and torch.equal(a.phi, c.phi)
