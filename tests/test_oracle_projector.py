"""Pins of the oracle's Joseph projector R_l and its transpose (CPU only).

R_l is the parallel-beam forward model evaluated on the level-l grid
(Sec. 4.1, the operator "R_i" of eq. (CT_sketches)).  What pins it:
  * closed-form chord lengths of an off-centre disk (first-order convergence;
    the off-centre position fixes the orientation of angles and axes);
  * exactness on affine images (linear interpolation plus the midpoint rule
    are exact for linear integrands), on every level;
  * theta = 0 and theta = pi/2 reduce to column and row sums;
  * the dot-product test and the explicit matrix, which tie the scatter
    transpose to the forward map entry by entry.
"""
import numpy as np
import pytest

import oracle
import synth


def _exact_disk(n, n_angles, n_det, rho, cx, cy):
    th = synth.angles_uniform(n_angles)[:, None]
    s = synth.detector_centres(n, n_det)[None, :]
    sp = s - (cx * np.cos(th) + cy * np.sin(th))
    return 2.0 * np.sqrt(np.maximum(rho * rho - sp * sp, 0.0)), sp


def test_disk_chords_converge_first_order():
    cx, cy, rho = 0.21, -0.13, 0.5
    means = []
    for n in (64, 128, 256, 512):
        g = oracle.Geometry(n, 12, 3 * n // 2)
        sino = oracle.project(g, 0, synth.disk_image(n, rho, cx, cy))
        exact, sp = _exact_disk(n, 12, 3 * n // 2, rho, cx, cy)
        th = synth.angles_uniform(12)[:, None]
        step = (2.0 / n) / np.maximum(np.abs(np.cos(th)), np.abs(np.sin(th)))
        err = np.abs(sino - exact)
        interior = np.abs(sp) <= 0.9 * rho
        assert (err / step)[interior].max() < 2.0, n
        means.append(err.mean())
    ratios = np.array(means[1:]) / np.array(means[:-1])
    assert ratios.max() < 0.65, ratios
    assert means[-1] / means[0] < 0.2


@pytest.mark.parametrize("lvl", [0, 1, 2])
def test_affine_images_are_exact(lvl):
    n, n_angles, n_det = 64, 30, 96
    alpha, beta, gamma = 0.7, -0.45, 0.3
    g = oracle.Geometry(n, n_angles, n_det)
    nl = n >> lvl
    h = 2.0 / nl
    z = synth.affine_image(nl, alpha, beta, gamma)
    sino = oracle.project(g, lvl, z)
    th = synth.angles_uniform(n_angles)
    s = synth.detector_centres(n, n_det)
    c0 = -1.0 + 0.5 * h
    checked = 0
    for a, t in enumerate(th):
        rows = 4 * a <= n_angles or 4 * a >= 3 * n_angles
        ct, st = np.cos(t), np.sin(t)
        ends = np.array([c0, -c0])
        for b, sb in enumerate(s):
            if rows:
                u = ((sb - ends * st) / ct - c0) / h
                expect = 2.0 * (alpha * sb / ct + gamma) / abs(ct)
            else:
                u = ((sb - ends * ct) / st - c0) / h
                expect = 2.0 * (beta * sb / st + gamma) / abs(st)
            if u.min() >= 0.0 and u.max() <= nl - 1:
                assert abs(sino[a, b] - expect) <= 1e-12 * max(1.0, abs(expect)), (a, b)
                checked += 1
    assert checked > n_angles * 10


def test_axis_angles_reduce_to_column_and_row_sums():
    n, n_angles, n_det = 32, 8, 48  # n_det - n even: bins sit on pixel centres
    g = oracle.Geometry(n, n_angles, n_det)
    z = synth.random_image(n, 3)
    sino = oracle.project(g, 0, z)
    h = 2.0 / n
    off = (n_det - n) // 2
    np.testing.assert_allclose(sino[0, off:off + n], h * z.sum(axis=0), rtol=0, atol=1e-12)
    a90 = n_angles // 2  # theta = pi/2: rays y = s cross rows
    np.testing.assert_allclose(sino[a90, off:off + n], h * z.sum(axis=1), rtol=0, atol=1e-12)
    # rays outside the image see nothing
    assert np.all(sino[0, :off - 1] == 0.0) and np.all(sino[0, off + n + 1:] == 0.0)


@pytest.mark.parametrize("lvl", [0, 1, 2, 3])
def test_dot_product(lvl):
    g = oracle.Geometry(64, 90, 92)
    nl = 64 >> lvl
    rng = np.random.default_rng(lvl)
    x = rng.standard_normal((nl, nl))
    y = rng.standard_normal((90, 92))
    lhs = np.vdot(oracle.project(g, lvl, x), y)
    rhs = np.vdot(x, oracle.backproject(g, lvl, y))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(x * x) * np.sum(y * y)) * 8


@pytest.mark.parametrize("lvl", [0, 1, 2])
def test_explicit_matrix_transpose_is_bitwise(lvl):
    g = oracle.Geometry(8, 6, 12)
    nl = 8 >> lvl
    A = oracle.dense_matrix(lambda e: oracle.project(g, lvl, e), (nl, nl), 6 * 12)
    At = oracle.dense_matrix(lambda e: oracle.backproject(g, lvl, e), (6, 12), nl * nl)
    assert np.array_equal(A, At.T)
    assert np.count_nonzero(A) > 0
    # each sample touches at most two pixels of its row/column: no ray sees a
    # pixel twice, so every entry is a single weight in (0, h_l/|cos|]
    assert A.max() <= (2.0 / nl) * np.sqrt(2.0) + 1e-15


def test_sample_count_bounded():
    g = oracle.Geometry(64, 90, 92)
    for lvl in range(3):
        c = oracle.count_samples(g, lvl)
        assert 0 < c <= 90 * 92 * (64 >> lvl)
