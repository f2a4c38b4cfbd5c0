"""GPU parity of the fan-beam projector pair and of Alg. 1 on fan geometries
against the FP64 oracle (through the C ABI).

Geometries: a 64^2 grid with 60 views over [0, 2pi); a ragged 48^2 grid with
37 listed views, an offset detector and a wide fan (rays of one view step
along rows and along columns); a 256^2 grid with 360 views x 384 bins at
levels 0-3; a 16^2 grid; the largest grid and detector (16384^2, 8192 bins)
and 4096^2 with 5800 bins; degenerate sizes (a 4^2 grid, one bin, one view).
Tolerances as for the parallel pair: relative l2 <= 1e-5 for projections and
backprojections, the tiny matrices bitwise transposed, iterates within 1e-4
(TV prior 1e-3) after 12-40 iterations.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, elementwise_ok, f32, host, max_rel, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu

# (n, views, bins, extent, source distance, detector distance, offset, listed views seed)
FANS = [(64, 60, 96, 1.0, 3.0, 2.0, 0.0, None), (48, 37, 71, 1.3, 2.9, 1.1, 0.07, 4),
        (256, 360, 384, 1.0, 4.0, 2.0, 0.0, None), (16, 8, 20, 1.0, 2.5, 0.5, -0.03, None)]


def _geoms(case):
    n, nv, nd, E, D, Dd, off, seed = case
    ang = None if seed is None else tuple(synth.angles_random(nv, seed))
    g = pk.Geometry(n, nv, nd, det_offset=off, extent=E, angles=ang, src_dist=D, det_dist=Dd)
    og = oracle.Geometry(n, nv, nd, s0=off, extent=E, angles=ang, src_dist=D, det_dist=Dd)
    return g, og


def _levels_for(n):
    return [l for l in range(4) if (n >> l) >= 2 and n % (1 << l) == 0]


@pytest.mark.parametrize("case", FANS)
def test_fan_project_and_backproject_match_oracle(case):
    g, og = _geoms(case)
    n, nv, nd = case[:3]
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 1))
    y = f32(synth.random_sinogram(nv, nd, 5))
    for l in _levels_for(n):
        say(f"fan {case[:3]} level {l}")
        got = host(pk.project(g, l, dev(x), work))
        exp = oracle.project(og, l, oracle.restrict(x, l))
        assert rel(got, exp) <= 1e-5, (case, l, rel(got, exp))
        got = host(pk.backproject(g, l, dev(y), work))
        exp = oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l
        assert rel(got, exp) <= 1e-5, (case, l, rel(got, exp))


@pytest.mark.parametrize("case", FANS[:2])
def test_fan_gpu_dot_product(case):
    g, _ = _geoms(case)
    n, nv, nd = case[:3]
    work = pk.workspace(g)
    rng = np.random.default_rng(3)
    for l in _levels_for(n):
        x = rng.standard_normal((n, n)).astype(np.float32)
        y = rng.standard_normal((nv, nd)).astype(np.float32)
        ax = host(pk.project(g, l, dev(x), work))
        aty = host(pk.backproject(g, l, dev(y), work))
        lhs, rhs = np.vdot(ax, y), np.vdot(x.astype(np.float64), aty)
        assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(ax) * np.linalg.norm(y), (l, lhs, rhs)


# (source distance, detector distance, spacing): a wide fan, where rays are
# dense and the transpose gathers, and a distant source with one-pixel bins,
# where it scatters on levels 0 and 1 (2 and 4 phases) and gathers on level 2
TINY = [(2.3, 0.9, 0.0), (6.0, 0.5, 0.25)]


@pytest.mark.parametrize("lvl", [0, 1, 2])
@pytest.mark.parametrize("tiny", TINY)
def test_fan_explicit_matrix_tiny(lvl, tiny):
    """An 8^2 grid: the GPU transpose realises the GPU forward's matrix
    transposed, bit for bit, and both the oracle's."""
    n, nv, nd = 8, 6, 14
    D, Dd, ds = tiny
    g = pk.Geometry(n, nv, nd, det_spacing=ds, det_offset=0.02, src_dist=D, det_dist=Dd)
    og = oracle.Geometry(n, nv, nd, ds=ds, s0=0.02, src_dist=D, det_dist=Dd)
    work = pk.workspace(g)
    A_gpu = np.empty((nv * nd, n * n))
    for q in range(n * n):
        e = np.zeros((n, n), dtype=np.float32)
        e.flat[q] = 1.0
        A_gpu[:, q] = host(pk.project(g, lvl, dev(e), work)).ravel()
    At_gpu = np.empty((n * n, nv * nd))
    for q in range(nv * nd):
        e = np.zeros((nv, nd), dtype=np.float32)
        e.flat[q] = 1.0
        At_gpu[:, q] = host(pk.backproject(g, lvl, dev(e), work)).ravel()
    assert np.array_equal(A_gpu, At_gpu.T)
    A_orc = oracle.dense_matrix(lambda z: oracle.project(og, lvl, oracle.restrict(z, lvl)), (n, n), nv * nd)
    assert np.count_nonzero(A_orc) > 0
    np.testing.assert_allclose(A_gpu, A_orc, rtol=0, atol=1e-6 * np.abs(A_orc).max())


@pytest.mark.parametrize("mode", [pk.FULL_PAPER, pk.FULL_UNBIASED])
def test_imask_on_fan_beam_matches_oracle(mode):
    g, og = _geoms(FANS[0])
    n, nv, nd = FANS[0][:3]
    b = f32(synth.random_sinogram(nv, nd, 30)) * 0.5 + 1.0
    log2f, p = (0, 1, 2), (0.4, 0.3, 0.3)
    sigma, iters = 0.02, 40
    say(f"imask fan mode {mode}")
    ost = oracle.imask_run(og, oracle.Levels(list(log2f), list(p), mode), oracle.Reg(lam=0.5), sigma, 42, 0, b, iters)
    prob = pk.Problem(g, pk.Levels(log2f, p, mode), pk.Regularizer(pk.REG_TIKHONOV, 0.5), pk.Params(sigma, 42, 0),
                      dev(b))
    prob.step(iters)
    assert prob.epochs == ost.epochs
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
    assert rel(host(prob.psi), ost.psi) <= 1e-4


def test_fan_beam_with_the_paper_prior_and_sequential_schedule():
    g, og = _geoms(FANS[1])
    n, nv, nd = FANS[1][:3]
    b = f32(synth.random_sinogram(nv, nd, 40)) * 0.3 + 0.5
    lv = (0, 1, 2)
    say("fan, Seq + TV prior")
    ost = oracle.imask_seq_run(og, oracle.Levels(list(lv), [0.5, 0.3, 0.2]),
                               oracle.Reg(oracle.REG_TV, lam=1e-2, tv_weight=2e-3, tv_inner=8), 5e-3, 1.0, 42, 0, b, 30)
    prob = pk.Problem(g, pk.Levels(lv, (0.5, 0.3, 0.2)), pk.Regularizer(pk.REG_TV, 1e-2, 2e-3, 0.0, 8),
                      pk.Params(5e-3, 42, 0, pk.SCHEDULE_SEQUENTIAL, 1.0), dev(b))
    prob.step(30)
    assert prob.epochs == ost.epochs
    assert host(prob.x_cur).min() >= 0.0
    assert rel(host(prob.x_cur), ost.x) <= 1e-3
    assert rel(host(prob.xbar), ost.xbar) <= 1e-3
    assert rel(host(prob.y_cur), ost.y) <= 1e-3


def test_fan_beam_batched_equals_alone_and_repeat_is_bitwise():
    g, _ = _geoms(FANS[0])
    n, nv, nd = FANS[0][:3]
    lv = pk.Levels((0, 1, 2), (0.4, 0.3, 0.3))
    mk = lambda s: pk.Problem(g, lv, pk.Regularizer(pk.REG_TIKHONOV, 0.5), pk.Params(0.02, 42, s),  # noqa: E731
                              dev(f32(synth.random_sinogram(nv, nd, 50 + s))))
    alone = [mk(s) for s in range(3)]
    for p in alone:
        p.step(15)
    batch = [mk(s) for s in range(3)]
    pk.step_many(batch, 15)
    for a, c in zip(alone, batch):
        assert np.array_equal(host(a.x_cur), host(c.x_cur)) and np.array_equal(host(a.y_cur), host(c.y_cur))


@pytest.mark.parametrize("D", [2.5, 6.0])
@pytest.mark.parametrize("n,nv,nd", [(4096, 6, 5800), (16384, 2, 8192)])
def test_fan_very_large_grids(n, nv, nd, D):
    """The largest grid and detector the boundary takes, levels 0 and 1; the
    transpose gathers at D = 2.5 and scatters at D = 6 (one wavefront of
    two rows per workgroup at 16384^2)."""
    g = pk.Geometry(n, nv, nd, src_dist=D, det_dist=0.5)
    og = oracle.Geometry(n, nv, nd, src_dist=D, det_dist=0.5)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 23))
    y = f32(synth.random_sinogram(nv, nd, 24))
    for l in (0, 1):
        say(f"fan grid {n} level {l}")
        got = host(pk.project(g, l, dev(x), work))
        assert rel(got, oracle.project(og, l, oracle.restrict(x, l))) <= 1e-5
        got = host(pk.backproject(g, l, dev(y), work))
        assert rel(got, oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l) <= 1e-5
    del work
    torch.cuda.empty_cache()


def test_fan_degenerate_sizes():
    """The smallest grid (4 x 4, levels 4 and 2), a single detector bin (the
    central ray) and a single view, 12 iterations of Alg. 1 (UNBIASED)."""
    for n, nv, nd, lv in ((4, 3, 5, (0, 1)), (16, 1, 1, (0, 1, 2)), (8, 7, 1, (0,))):
        g = pk.Geometry(n, nv, nd, src_dist=2.5, det_dist=0.5)
        og = oracle.Geometry(n, nv, nd, src_dist=2.5, det_dist=0.5)
        b = f32(synth.random_sinogram(nv, nd, 60 + n))
        p = (1.0 / len(lv),) * len(lv)
        say(f"fan degenerate n={n} views={nv} bins={nd}")
        ost = oracle.imask_run(og, oracle.Levels(list(lv), list(p), oracle.MODE_UNBIASED), oracle.Reg(lam=0.5),
                               0.05, 42, 0, b, 12)
        prob = pk.Problem(g, pk.Levels(lv, p, pk.FULL_UNBIASED), pk.Regularizer(pk.REG_TIKHONOV, 0.5),
                          pk.Params(0.05, 42, 0), dev(b))
        prob.step(12)
        assert prob.epochs == ost.epochs
        assert rel(host(prob.x_cur), ost.x) <= 1e-4
        assert rel(host(prob.y_cur), ost.y) <= 1e-4


def test_fan_beam_with_compact_tables_and_independent_draws():
    g, og = _geoms(FANS[0])
    n, nv, nd = FANS[0][:3]
    b = f32(synth.random_sinogram(nv, nd, 41)) * 0.3 + 0.5
    lv, p = (0, 1, 2), (0.4, 0.3, 0.3)
    say("fan, compact tables")
    ost = oracle.imask_compact_run(og, oracle.Levels(list(lv), list(p)), oracle.Reg(lam=0.5), 0.02, 42, 0, b, 30)
    prob = pk.Problem(g, pk.Levels(lv, p), pk.Regularizer(pk.REG_TIKHONOV, 0.5), pk.Params(0.02, 42, 0), dev(b),
                      compact_tables=True)
    prob.step(30)
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
    say("fan, independent draws")
    ost = oracle.imask_indep_run(og, oracle.Levels(list(lv), list(p)), oracle.Reg(lam=0.5), 0.02, 42, 0, 5, b, 30)
    prob = pk.Problem(g, pk.Levels(lv, p), pk.Regularizer(pk.REG_TIKHONOV, 0.5),
                      pk.Params(0.02, 42, 0, draw_mode=pk.DRAW_INDEPENDENT, dual_stream_id=5), dev(b))
    prob.step(30)
    assert prob.epochs == ost.epochs
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4


def test_fan_bench_workload():
    """The fan workload bench.py --fan times (512^2, 720 views x 768 bins,
    source 4, detector 2, data along the fan's rays, smoothed TV, PAPER,
    four levels): the projector pair within 1e-5 at every level (the
    transpose scatters on levels 0 and 1, with four and two rays per trip,
    and gathers on levels 2 and 3), then 21 iterations of Alg. 1 within
    1e-3, launched as the benchmark launches them."""
    n, nv, nd = 512, 720, 768
    g = pk.Geometry(n, nv, nd, src_dist=4.0, det_dist=2.0)
    og = oracle.Geometry(n, nv, nd, src_dist=4.0, det_dist=2.0)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 31))
    y = f32(synth.random_sinogram(nv, nd, 32))
    for l in range(4):
        say(f"fan bench geometry level {l}")
        got = host(pk.project(g, l, dev(x), work))
        exp = oracle.project(og, l, oracle.restrict(x, l))
        assert rel(got, exp) <= 1e-5, l
        # element by element within the FP32 bound of each ray's 2 N_l taps
        # (and the 4^l-term block mean)
        absref = oracle.project(og, l, oracle.restrict(np.abs(x), l))
        ok, worst = elementwise_ok(got, exp, absref, 2 * (n >> l) + 16 + 4 ** l)
        assert ok, ("forward", l, worst)
        assert max_rel(got, exp) <= 1e-5, ("forward", l, max_rel(got, exp))
        say(f"  level {l} forward: worst element at {worst:.2e} of its bound, max_rel {max_rel(got, exp):.2e}")
        got = host(pk.backproject(g, l, dev(y), work))
        exp = oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l
        assert rel(got, exp) <= 1e-5, l
        # a pixel takes two taps from each of at most 2^l (D + Dd)/(D - 1.6)
        # + 1 rays per view (rays at least a magnified pixel apart at the
        # detector), then up to 2048 partial images in order
        absref = oracle.prolong(oracle.backproject(og, l, np.abs(y)), l) / 4 ** l
        ok, worst = elementwise_ok(got, exp, absref, 2 * nv * (3 * 2 ** l + 2) + 2048)
        assert ok, ("transpose", l, worst)
        assert max_rel(got, exp) <= 1e-5, ("transpose", l, max_rel(got, exp))
        say(f"  level {l} transpose: worst element at {worst:.2e} of its bound, max_rel {max_rel(got, exp):.2e}")
    _, b = synth.fan_ct_problem(n, nv, nd, 4.0, 2.0, 1e5, 1000, 2000)
    b = f32(b)
    reg_o = oracle.Reg(oracle.REG_SMOOTH_TV, lam=1e-3, tv_weight=2e-4, tv_eps=1e-3, tv_inner=10)
    reg_g = pk.Regularizer(pk.REG_SMOOTH_TV, 1e-3, 2e-4, 1e-3, 10)
    say("fan bench workload, 21 iterations")
    ost = oracle.imask_run(og, oracle.Levels([0, 1, 2, 3], [0.25] * 4), reg_o, 1e-3, 42, 0, b, 21)
    prob = pk.Problem(g, pk.Levels.uniform((0, 1, 2, 3), pk.FULL_PAPER), reg_g, pk.Params(1e-3, 42, 0), dev(b))
    prob.step(21)
    assert prob.epochs == ost.epochs > 10.0
    assert rel(host(prob.x_cur), ost.x) <= 1e-3
    assert rel(host(prob.y_cur), ost.y) <= 1e-3
    assert max_rel(host(prob.x_cur), ost.x) <= 3e-3
    assert max_rel(host(prob.y_cur), ost.y) <= 3e-3


@pytest.mark.parametrize("case,S,iters", [(0, 4, 40), (2, 3, 16)])
def test_fan_beam_with_measurement_blocks(case, S, iters):
    """Image sketches with S blocks of contiguous views (reading 24 on a fan
    beam) against the oracle, both modes: the 64^2 geometry (scatter with
    two rays per trip at level 0, gather above) and the 256^2 one (four rays
    per trip at level 0)."""
    g, og = _geoms(FANS[case])
    n, nv, nd = FANS[case][:3]
    b = f32(synth.random_sinogram(nv, nd, 70 + case)) * 0.5 + 1.0
    log2f, p = (0, 1, 2), (0.4, 0.3, 0.3)
    for mode in (pk.FULL_PAPER, pk.FULL_UNBIASED):
        say(f"fan blocks case {case} S={S} mode {mode}")
        ost = oracle.imask_blocks_run(og, oracle.Levels(list(log2f), list(p), mode), oracle.Reg(lam=0.5), 0.02, 42,
                                      0, S, b, iters)
        prob = pk.Problem(g, pk.Levels(log2f, p, mode, S), pk.Regularizer(pk.REG_TIKHONOV, 0.5),
                          pk.Params(0.02, 42, 0), dev(b))
        prob.step(iters)
        assert prob.epochs == pytest.approx(ost.epochs, rel=1e-12)
        assert rel(host(prob.x_cur), ost.x) <= 1e-4
        assert rel(host(prob.y_cur), ost.y) <= 1e-4
        assert rel(host(prob.psi), ost.psi) <= 1e-4
