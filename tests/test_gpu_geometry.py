"""GPU parity of the projector pair and of Alg. 1 on listed angles (any real
theta, any order) and a domain [-E, E]^2, against the FP64 oracle.

Detector spacings and offsets other than the defaults ride along.  Same bars
as the default geometry: relative l2 <= 1e-5 for projections and
backprojections, an exact (bitwise) transpose on a tiny grid, 1e-4 for x and
y after a run of Alg. 1; a listed copy of the default angles reproduces the
default geometry bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, f32, host, rel, say

import paper_2412_10249_amd as pk

pytestmark = pytest.mark.gpu

# (n, n_det, angles, extent, spacing in pixels, offset / E): full circle,
# limited angle, unsorted with repeats and negative values, and a case
# spanning several forward bands; spacings and offsets off the defaults
CASES = [
    (64, 92, tuple(synth.angles_random(40, 1)), 2.3, 1.0, 0.0),
    (48, 71, tuple(synth.angles_random(13, 2, 0.0, 2.0 * np.pi / 3)), 1.0, 0.7, 0.15),
    (32, 50, (0.0, -0.3, 2.9, 0.0, 7.1, np.pi / 4, 3 * np.pi / 4, np.pi / 2), 0.6, 1.6, -0.4),
    (256, 300, tuple(synth.angles_random(97, 3)), 1.7, 1.25, 0.05),
]


def _geoms(n, nd, ang, E, spacing_px=1.0, offset=0.0):
    ds, s0 = spacing_px * 2.0 * E / n, offset * E
    return (pk.Geometry(n, len(ang), nd, ds, s0, extent=E, angles=ang),
            oracle.Geometry(n, len(ang), nd, ds, s0, extent=E, angles=ang))


def _levels_for(n):
    return [l for l in range(4) if (n >> l) >= 2 and n % (1 << l) == 0]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_listed_project_and_backproject_match_oracle(case):
    n, nd, ang, E, sp, off = CASES[case]
    g, og = _geoms(n, nd, ang, E, sp, off)
    work = pk.workspace(g)
    x = f32(synth.random_image(n, 10 + case))
    y = f32(synth.random_sinogram(len(ang), nd, 20 + case))
    for l in _levels_for(n):
        say(f"listed case {case} level {l}")
        got = host(pk.project(g, l, dev(x), work))
        exp = oracle.project(og, l, oracle.restrict(x, l))
        assert rel(got, exp) <= 1e-5, (case, l, rel(got, exp))
        got = host(pk.backproject(g, l, dev(y), work))
        exp = oracle.prolong(oracle.backproject(og, l, y), l) / 4 ** l
        assert rel(got, exp) <= 1e-5, (case, l, rel(got, exp))


@pytest.mark.parametrize("lvl", [0, 1])
def test_listed_explicit_matrix_tiny(lvl):
    n, nd = 8, 12
    ang = tuple(synth.angles_random(6, 7))
    g, og = _geoms(n, nd, ang, 0.8)
    work = pk.workspace(g)
    na = len(ang)
    A = np.empty((na * nd, n * n))
    for q in range(n * n):
        e = np.zeros((n, n), dtype=np.float32)
        e.flat[q] = 1.0
        A[:, q] = host(pk.project(g, lvl, dev(e), work)).ravel()
    At = np.empty((n * n, na * nd))
    for q in range(na * nd):
        e = np.zeros((na, nd), dtype=np.float32)
        e.flat[q] = 1.0
        At[:, q] = host(pk.backproject(g, lvl, dev(e), work)).ravel()
    assert np.array_equal(A, At.T)
    A_orc = oracle.dense_matrix(lambda z: oracle.project(og, lvl, oracle.restrict(z, lvl)), (n, n), na * nd)
    np.testing.assert_allclose(A, A_orc, rtol=0, atol=1e-6 * np.abs(A_orc).max())


def test_listed_default_angles_are_bitwise_the_default():
    n, na, nd = 64, 90, 92  # 90 angles: none at exactly 45 or 135 degrees
    g0 = pk.Geometry(n, na, nd)
    g1 = pk.Geometry(n, na, nd, angles=tuple(synth.angles_uniform(na)))
    w0, w1 = pk.workspace(g0), pk.workspace(g1)
    x = dev(synth.random_image(n, 4))
    y = dev(synth.random_sinogram(na, nd, 5))
    for l in (0, 1, 2):
        assert np.array_equal(host(pk.project(g0, l, x, w0)), host(pk.project(g1, l, x, w1)))
        assert np.array_equal(host(pk.backproject(g0, l, y, w0)), host(pk.backproject(g1, l, y, w1)))


def test_imask_on_listed_angles_matches_oracle():
    n, nd, E = 64, 96, 1.5
    ang = tuple(synth.angles_random(50, 9, 0.0, np.pi))
    g, og = _geoms(n, nd, ang, E)
    b = f32(synth.random_sinogram(len(ang), nd, 30)) * 0.5 + 1.0
    log2f, p = (0, 1, 2), (0.4, 0.3, 0.3)
    sigma, iters = 0.02, 40
    say("imask listed angles")
    ost = oracle.imask_run(og, oracle.Levels(list(log2f), list(p)), oracle.Reg(lam=0.5), sigma, 42, 0, b, iters)
    prob = pk.Problem(g, pk.Levels(log2f, p), pk.Regularizer(pk.REG_TIKHONOV, 0.5), pk.Params(sigma, 42, 0), dev(b))
    prob.step(iters)
    assert prob.epochs == ost.epochs
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4


def test_listed_angles_with_the_paper_prior_and_sequential_schedule():
    """ImaSk-Seq with the TV + nonnegativity prior on a limited-angle listed
    geometry with a shifted, finer detector: x, xbar, y, dual pair within 1e-3."""
    n, nd, E = 64, 110, 1.2
    ang = tuple(synth.angles_random(45, 12, 0.2, 2.6))
    g, og = _geoms(n, nd, ang, E, 0.8, 0.1)
    b = f32(synth.random_sinogram(len(ang), nd, 40)) * 0.3 + 0.5
    lv = (0, 1, 2)
    say("listed angles, Seq + TV prior")
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
    assert rel(host(prob.tvd[prob.cur]), ost.tvd) <= 1e-3


def test_listed_angles_with_compact_tables_and_independent_draws():
    n, nd = 48, 70
    ang = tuple(synth.angles_random(33, 13))
    g, og = _geoms(n, nd, ang, 1.0)
    b = f32(synth.random_sinogram(len(ang), nd, 41)) * 0.3 + 0.5
    lv, p = (0, 1, 2), (0.4, 0.3, 0.3)
    say("listed angles, compact tables")
    ost = oracle.imask_compact_run(og, oracle.Levels(list(lv), list(p)), oracle.Reg(lam=0.5), 0.02, 42, 0, b, 30)
    prob = pk.Problem(g, pk.Levels(lv, p), pk.Regularizer(pk.REG_TIKHONOV, 0.5), pk.Params(0.02, 42, 0), dev(b),
                      compact_tables=True)
    prob.step(30)
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
    say("listed angles, independent draws")
    ost = oracle.imask_indep_run(og, oracle.Levels(list(lv), list(p)), oracle.Reg(lam=0.5), 0.02, 42, 0, 5, b, 30)
    prob = pk.Problem(g, pk.Levels(lv, p), pk.Regularizer(pk.REG_TIKHONOV, 0.5),
                      pk.Params(0.02, 42, 0, draw_mode=pk.DRAW_INDEPENDENT, dual_stream_id=5), dev(b))
    prob.step(30)
    assert prob.epochs == ost.epochs
    assert rel(host(prob.x_cur), ost.x) <= 1e-4
    assert rel(host(prob.y_cur), ost.y) <= 1e-4
