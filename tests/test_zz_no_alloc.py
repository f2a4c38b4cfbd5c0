"""The workspace-free transpose (imask_backproject_noalloc) against
imask_backproject with a prepared workspace, through the C ABI: equal bit
for bit on two calls in a row, the second on a smaller geometry (the static
array keeps the first call's contents), and within the projector tolerance
of the oracle's scatter transpose."""
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, say

import paper_2412_10249_amd as pk
from paper_2412_10249_amd import imask as im

pytestmark = pytest.mark.gpu

CASES = [((512, 720, 768), 0), ((64, 90, 92), 1), ((512, 720, 768), 2)]


def _pair(shape, lvl, seed):
    g = pk.Geometry(*shape)
    y = dev(synth.random_sinogram(shape[1], shape[2], seed))
    work = pk.workspace(g)
    ref = im.backproject(g, lvl, y, work)
    out = torch.full(g.image_shape, float("nan"), device="cuda")
    im.backproject_noalloc(g, lvl, y, out)
    torch.cuda.synchronize()
    return g, y, ref, out


def test_noalloc_equals_backproject_twice_in_a_row():
    for q, (shape, lvl) in enumerate(CASES):
        say(f"noalloc transpose {shape} level {lvl}")
        g, y, ref, out = _pair(shape, lvl, 70 + q)
        assert torch.equal(out, ref), (shape, lvl)
        og = oracle.Geometry(*shape)
        if lvl == 0:
            exp = oracle.backproject(og, 0, host(y))
        else:
            exp = oracle.sketch_adj(og, oracle.Levels([0, lvl], [0.5, 0.5]), 1, host(y))
        assert rel(host(out), exp) <= 1e-5

