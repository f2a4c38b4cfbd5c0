"""GPU parity of the projector pair, resampling and sketched operators
against the FP64 oracle (through the C ABI).

Tolerances: relative l2 <= 1e-5 for projections and backprojections (FP32
coordinates and sums against FP64); the GPU pair is an exact transpose, so
the matrices it realises on a tiny grid agree bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, elementwise_ok, f32, host, max_rel, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu

GEOMS = [(64, 90, 92), (48, 37, 71), (16, 8, 20), (32, 1, 50), (128, 180, 192)]


def _levels_for(n):
    l, out = 0, []
    while l <= 3 and (n >> l) >= 2 and n % (1 << l) == 0:
        out.append(l)
        l += 1
    return out


@pytest.mark.parametrize("geom", GEOMS)
def test_project_matches_oracle(geom):
    n, na, nd = geom
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    for seed, img in ((0, synth.random_image(n, 1)), (1, synth.ct_problem(n, na, nd, 1e4, 1000, 2000)[0])):
        x = f32(img)
        for l in _levels_for(n):
            say(f"project {geom} level {l} input {seed}")
            got = host(pk.project(g, l, dev(x), work))
            exp = oracle.project(og, l, oracle.restrict(x, l))
            assert rel(got, exp) <= 1e-5, (geom, l, rel(got, exp))


@pytest.mark.parametrize("geom", GEOMS)
def test_backproject_matches_oracle(geom):
    n, na, nd = geom
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    y = f32(synth.random_sinogram(na, nd, 5))
    for l in _levels_for(n):
        say(f"backproject {geom} level {l}")
        got = host(pk.backproject(g, l, dev(y), work))
        exp = oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l
        assert rel(got, exp) <= 1e-5, (geom, l, rel(got, exp))


@pytest.mark.parametrize("geom", GEOMS[:3])
def test_gpu_dot_product(geom):
    n, na, nd = geom
    g = pk.Geometry(n, na, nd)
    work = pk.workspace(g)
    rng = np.random.default_rng(3)
    for l in _levels_for(n):
        x = rng.standard_normal((n, n)).astype(np.float32)
        y = rng.standard_normal((na, nd)).astype(np.float32)
        ax = host(pk.project(g, l, dev(x), work))
        aty = host(pk.backproject(g, l, dev(y), work))
        lhs, rhs = np.vdot(ax, y), np.vdot(x.astype(np.float64), aty)
        assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(ax) * np.linalg.norm(y), (l, lhs, rhs)


@pytest.mark.parametrize("n,lvl", [(8, 0), (8, 1), (8, 2), (16, 3)])
def test_explicit_matrix_tiny(n, lvl):
    # level 3 of a 16^2 grid has rays 6-8 bins per pixel: the transpose's run form
    na, nd = 6, 12 * n // 8
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    A_gpu = np.empty((na * nd, n * n))
    for q in range(n * n):
        e = np.zeros((n, n), dtype=np.float32)
        e.flat[q] = 1.0
        A_gpu[:, q] = host(pk.project(g, lvl, dev(e), work)).ravel()
    At_gpu = np.empty((n * n, na * nd))
    for q in range(na * nd):
        e = np.zeros((na, nd), dtype=np.float32)
        e.flat[q] = 1.0
        At_gpu[:, q] = host(pk.backproject(g, lvl, dev(e), work)).ravel()
    # the transpose recomputes the forward's weights: an exact transpose
    assert np.array_equal(A_gpu, At_gpu.T)
    A_orc = oracle.dense_matrix(lambda z: oracle.project(og, lvl, oracle.restrict(z, lvl)), (n, n), na * nd)
    np.testing.assert_allclose(A_gpu, A_orc, rtol=0, atol=1e-6 * np.abs(A_orc).max())


def test_resample_modes():
    n = 64
    x = f32(synth.random_image(n, 8))
    lv = pk.Levels((0, 1, 2, 3), (0.4, 0.3, 0.2, 0.1))
    olv = oracle.Levels([0, 1, 2, 3], [0.4, 0.3, 0.2, 0.1])
    for l in (1, 2, 3):
        got = host(pk.resample(dev(x), l, pk.RESTRICT))
        np.testing.assert_allclose(got, oracle.restrict(x, l), rtol=0, atol=2e-7)
        z = f32(synth.random_image(n >> l, 9))
        np.testing.assert_allclose(host(pk.resample(dev(z), l, pk.PROLONG)), oracle.prolong(z, l), rtol=0, atol=0)
        np.testing.assert_allclose(host(pk.resample(dev(z), l, pk.RESTRICT_ADJ)), oracle.prolong(z, l) / 4 ** l,
                                   rtol=0, atol=1e-9)
        np.testing.assert_allclose(host(pk.resample(dev(x), l, pk.PROJECT)),
                                   oracle.prolong(oracle.restrict(x, l), l), rtol=0, atol=2e-7)
    got = host(pk.resample(dev(x), 0, pk.COMPENSATE, lv))
    np.testing.assert_allclose(got, oracle.compensate(x, olv), rtol=0, atol=1e-5)


@pytest.mark.parametrize("mode", [pk.FULL_PAPER, pk.FULL_UNBIASED])
def test_sketch_operators_match_oracle(mode):
    n, na, nd = 64, 45, 96
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    lv = pk.Levels((0, 1, 3), (0.5, 0.3, 0.2), mode)
    olv = oracle.Levels([0, 1, 3], [0.5, 0.3, 0.2], mode)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 4))
    y = f32(synth.random_sinogram(na, nd, 6))
    for k in range(3):
        say(f"sketch mode {mode} k {k}")
        got = host(pk.sketch_apply(g, lv, k, dev(x), False, work))
        assert rel(got, oracle.sketch_fwd(og, olv, k, x)) <= 1e-5
        got = host(pk.sketch_apply(g, lv, k, dev(y), True, work))
        assert rel(got, oracle.sketch_adj(og, olv, k, y)) <= 1e-5


def test_full_size_projector_pair():
    """720 angles x 768 bins on a 512^2 grid, every level (the race workload)."""
    n, na, nd = 512, 720, 768
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    x = f32(synth.ct_problem(n, na, nd, 1e5, 1000, 2000)[0])
    y = f32(synth.random_sinogram(na, nd, 11))
    for l in range(4):
        say(f"full-size level {l}")
        _pair_elementwise(g, og, work, l, x, y)


def _pair_elementwise(g, og, work, l, x, y, extra_terms=0):
    """Projector pair at level l: relative l2 <= 1e-5 and, element by
    element, within the FP32 rounding bound of each sum (forward: a ray's
    2 N_l taps, band partials and the 4^l-term block mean; transpose: up to
    four taps per angle and pixel, and the ordered partial-image sum)."""
    nl = g.n >> l
    got = host(pk.project(g, l, dev(x), work))
    exp = oracle.project(og, l, oracle.restrict(x, l))
    assert rel(got, exp) <= 1e-5, (l, rel(got, exp))
    absref = oracle.project(og, l, oracle.restrict(np.abs(x), l))
    ok, worst = elementwise_ok(got, exp, absref, 2 * nl + 16 + 4 ** l + extra_terms)
    assert ok, ("forward", l, worst)
    assert max_rel(got, exp) <= 1e-5, ("forward", l, max_rel(got, exp))
    say(f"  level {l} forward: worst element at {worst:.2e} of its bound, max_rel {max_rel(got, exp):.2e}")
    got = host(pk.backproject(g, l, dev(y), work))
    exp = oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l
    assert rel(got, exp) <= 1e-5, (l, rel(got, exp))
    absref = oracle.prolong(oracle.backproject(og, l, np.abs(y)), l) / 4 ** l
    ok, worst = elementwise_ok(got, exp, absref, 4 * g.n_angles + 64 + extra_terms)
    assert ok, ("transpose", l, worst)
    assert max_rel(got, exp) <= 1e-5, ("transpose", l, max_rel(got, exp))
    say(f"  level {l} transpose: worst element at {worst:.2e} of its bound, max_rel {max_rel(got, exp):.2e}")


@pytest.mark.parametrize("n", [384, 768])
def test_batched_workload_sizes_projector_pair(n):
    """The mixed-size batch's other grids (angles = bins = 1.5 N), levels
    0-3, against the oracle element by element."""
    na = nd = 3 * n // 2
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    x = f32(synth.ct_problem(n, na, nd, 1e5, 1000 + n, 2000 + n)[0])
    y = f32(synth.random_sinogram(na, nd, 11 + n))
    for l in range(4):
        say(f"grid {n} level {l}")
        _pair_elementwise(g, og, work, l, x, y)


def test_large_grid_projector_pair():
    """1024^2 grid, 1536 angles x 1536 bins: the level-0 forward exceeds one
    LDS band (direct path) and the scatter stages two angles per batch."""
    n, na, nd = 1024, 1536, 1536
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 21))
    y = f32(synth.random_sinogram(na, nd, 22))
    for l in (0, 1):
        say(f"1024 grid level {l}")
        got = host(pk.project(g, l, dev(x), work))
        assert rel(got, oracle.project(og, l, oracle.restrict(x, l))) <= 1e-5
        got = host(pk.backproject(g, l, dev(y), work))
        assert rel(got, oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l) <= 1e-5


@pytest.mark.parametrize("n,na,nd", [(4096, 6, 5800), (8192, 3, 8192), (16384, 2, 8192)])
def test_very_large_grids(n, na, nd):
    """Rows longer than the LDS of the default transpose tile (a fallback tile
    of fewer rows), the direct forward, and the largest detector."""
    g = pk.Geometry(n, na, nd)
    og = oracle.Geometry(n, na, nd)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 23))
    y = f32(synth.random_sinogram(na, nd, 24))
    for l in (0, 1):
        say(f"grid {n} level {l}")
        got = host(pk.project(g, l, dev(x), work))
        assert rel(got, oracle.project(og, l, oracle.restrict(x, l))) <= 1e-5
        got = host(pk.backproject(g, l, dev(y), work))
        assert rel(got, oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l) <= 1e-5
    del work
    torch.cuda.empty_cache()


def test_projection_is_deterministic():
    g = pk.Geometry(128, 180, 192)
    work = pk.workspace(g)
    x = dev(synth.random_image(128, 2))
    y = dev(synth.random_sinogram(180, 192, 2))
    a1, a2 = pk.project(g, 0, x, work), pk.project(g, 0, x, work)
    b1, b2 = pk.backproject(g, 1, y, work), pk.backproject(g, 1, y, work)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


@pytest.mark.parametrize("n,na,nd", [(512, 720, 768), (96, 60, 150)])
def test_unbiased_full_sketch_in_a_step_matches_oracle(n, na, nd):
    """The UNBIASED full-resolution sketch K_0 = p_0^{-1}(R_0 - sum p_l R_l T_l)
    and its transpose as one step of Alg. 1 applies them (forward terms in
    one launch, the coarse transposes side by side in the partial-image
    buffer, one launch per tile shape): from x, y random and zero tables
    the first step (drawn sketch 0: stream 2) refreshes psi_0 = K_0 x and
    phi_0 = K_0^T y, compared with the oracle's sketches (l2 and element
    by element)."""
    levels = (0, 1, 2, 3)
    x = f32(synth.random_image(n, 51))
    y = f32(synth.random_sinogram(na, nd, 52))
    prob = pk.Problem(pk.Geometry(n, na, nd), pk.Levels.uniform(levels, pk.FULL_UNBIASED),
                      pk.Regularizer(pk.REG_TIKHONOV, 1e-2), pk.Params(1e-3, 42, 2), dev(np.zeros((na, nd))))
    assert int(pk.draws(prob.params, prob.levels, 0, 1)[0]) == 0
    prob.x[0].copy_(dev(x))
    prob.y[0].copy_(dev(y))
    say(f"UNBIASED full sketch in a step, {n}^2")
    prob.step(1)
    og = oracle.Geometry(n, na, nd)
    olv = oracle.Levels(list(levels), [0.25] * 4, oracle.MODE_UNBIASED)
    fwd = oracle.sketch_fwd(og, olv, 0, x)
    got = host(prob.psi[0])
    assert rel(got, fwd) <= 1e-5
    assert max_rel(got, fwd) <= 1e-5
    adj = oracle.sketch_adj(og, olv, 0, y)
    got = host(prob.phi_tables()[0])
    assert rel(got, adj) <= 1e-5
    assert max_rel(got, adj) <= 1e-5
