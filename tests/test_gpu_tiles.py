"""Tuned launch shapes (imask_set_tiles) keep the projector pair exact: for
every transpose tile, workgroup target and forward band budget the
autotuner may choose, the pair at every level of a 256^2 / 384 x 384
geometry matches the oracle (1e-5), the transpose stays the exact adjoint
(dot-product test), and a batched run under tuned tiles equals the same
problem run alone under them."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk
from paper_2412_10249_amd import autotune
from paper_2412_10249_amd.batch import Batch

pytestmark = pytest.mark.gpu

N, NA, ND = 256, 384, 384


@pytest.fixture(autouse=True)
def _reset_tiles():
    yield
    for l in range(4):
        autotune.reset_tiles(N >> l, NA, ND)


@pytest.mark.parametrize("shape", autotune.BP_SHAPES)
def test_every_tile_shape_matches_oracle(shape):
    g = pk.Geometry(N, NA, ND)
    og = oracle.Geometry(N, NA, ND)
    x = f32(synth.random_image(N, 41))
    y = f32(synth.random_sinogram(NA, ND, 42))
    work = pk.workspace(g)
    for wg, kb in ((512, 156), (2048, 0)):
        for l in range(4):
            autotune.set_tiles(N >> l, NA, ND, shape, wg, kb)
        for l in range(4):
            say(f"tiles {shape} wg {wg} fwd {kb} KB level {l}")
            got = host(pk.project(g, l, dev(x), work))
            assert rel(got, oracle.project(og, l, oracle.restrict(x, l))) <= 1e-5
            aty = host(pk.backproject(g, l, dev(y), work))
            assert rel(aty, oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l) <= 1e-5
            lhs, rhs = np.vdot(got, y), np.vdot(x, aty)
            assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(got) * np.linalg.norm(y)


def test_batch_under_tuned_tiles_equals_alone():
    for l in range(4):
        autotune.set_tiles(N >> l, NA, ND, (2, 4), 2048, 156)
    _, b = synth.ct_problem(N, NA, ND, 1e5, 1300, 2300)

    def mk(q):
        return pk.Problem(pk.Geometry(N, NA, ND), pk.Levels.uniform((0, 1, 2, 3), pk.FULL_UNBIASED),
                          pk.Regularizer(pk.REG_TIKHONOV, 1e-2), pk.Params(1e-3, 42, q), dev(b))
    batched = [mk(q) for q in range(3)]
    bt = Batch(batched, 10, pk.BUDGET_ITERS)
    bt.run(graph=True)
    bt.sync_state()
    for q, p in enumerate(batched):
        a = mk(q)
        a.step(10)
        torch.cuda.synchronize()
        assert torch.equal(a.x_cur, p.x_cur) and torch.equal(a.y_cur, p.y_cur) and a.epochs == p.epochs
