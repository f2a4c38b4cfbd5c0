"""Pins of the oracle's Joseph projector R_l and its transpose (CPU only).

R_l is the parallel-beam forward model evaluated on the level-l grid
(Sec. 4.1, the operator "R_i" of eq. (CT_sketches)).  What pins it:
  * closed-form chord lengths of an off-centre disk (first-order convergence;
    the off-centre position fixes the orientation of angles and axes);
  * exactness on affine images (linear interpolation plus the midpoint rule
    are exact for linear integrands), on every level;
  * theta = 0 and theta = pi/2 reduce to column and row sums;
  * the dot-product test and the explicit matrix, which tie the scatter
    transpose to the forward map entry by entry;
  * with a listed set of angles anywhere in [0, 2pi) and a domain [-E, E]^2:
    the disk chords and affine exactness again, bitwise agreement with the
    default angles when the list is the default one, and the mirror symmetry
    of opposite angles (theta + pi sees the detector reversed).
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


# ---- listed angles (any real theta) and a domain [-E, E]^2 ----

def _listed(n, n_det, seed, n_angles=16, extent=2.5):
    th = synth.angles_random(n_angles, seed)
    return oracle.Geometry(n, n_angles, n_det, extent=extent, angles=tuple(th)), th


def test_listed_angles_disk_chords_converge():
    E = 2.5
    cx, cy, rho = 0.21 * E, -0.13 * E, 0.5 * E
    means = []
    for n in (64, 128, 256, 512):
        g, th = _listed(n, 3 * n // 2, 11, extent=E)
        sino = oracle.project(g, 0, synth.disk_image(n, rho, cx, cy, extent=E))
        s = synth.detector_centres(n, 3 * n // 2, extent=E)[None, :]
        t = th[:, None]
        sp = s - (cx * np.cos(t) + cy * np.sin(t))
        exact = 2.0 * np.sqrt(np.maximum(rho * rho - sp * sp, 0.0))
        step = (2.0 * E / n) / np.maximum(np.abs(np.cos(t)), np.abs(np.sin(t)))
        err = np.abs(sino - exact)
        assert (err / step)[np.abs(sp) <= 0.9 * rho].max() < 2.0, n
        means.append(err.mean())
    ratios = np.array(means[1:]) / np.array(means[:-1])
    assert ratios.max() < 0.65, ratios


@pytest.mark.parametrize("lvl", [0, 1, 2])
def test_listed_angles_affine_images_are_exact(lvl):
    n, n_det, E = 64, 96, 1.7
    g, th = _listed(n, n_det, 5 + lvl, n_angles=40, extent=E)
    alpha, beta, gamma = 0.7, -0.45, 0.3
    nl = n >> lvl
    h = 2.0 * E / nl
    sino = oracle.project(g, lvl, synth.affine_image(nl, alpha, beta, gamma, extent=E))
    s = synth.detector_centres(n, n_det, extent=E)
    c0 = -E + 0.5 * h
    ends = np.array([c0, -c0])
    checked = 0
    for a, t in enumerate(th):
        ct, st = np.cos(t), np.sin(t)
        rows = abs(ct) >= abs(st)
        for b, sb in enumerate(s):
            if rows:
                u = ((sb - ends * st) / ct - c0) / h
                expect = 2.0 * E * (alpha * sb / ct + gamma) / abs(ct)
            else:
                u = ((sb - ends * ct) / st - c0) / h
                expect = 2.0 * E * (beta * sb / st + gamma) / abs(st)
            if u.min() >= 0.0 and u.max() <= nl - 1:
                assert abs(sino[a, b] - expect) <= 1e-12 * max(1.0, abs(expect)), (a, b)
                checked += 1
    assert checked > 40 * 10


def test_listed_uniform_angles_match_the_default_bitwise():
    # 30 angles: none at exactly 45 or 135 degrees, where the two stepping
    # rules may pick different (equally valid) axes
    g0 = oracle.Geometry(64, 30, 92)
    g1 = oracle.Geometry(64, 30, 92, angles=tuple(synth.angles_uniform(30)))
    z = synth.random_image(64, 2)
    y = synth.random_sinogram(30, 92, 3)
    for lvl in (0, 2):
        zl = z[:64 >> lvl, :64 >> lvl]
        assert np.array_equal(oracle.project(g0, lvl, zl), oracle.project(g1, lvl, zl))
        assert np.array_equal(oracle.backproject(g0, lvl, y), oracle.backproject(g1, lvl, y))


def test_opposite_angles_mirror_the_detector():
    # theta + pi is the same line set with s -> -s; bins symmetric about 0
    th = synth.angles_random(12, 8, 0.0, np.pi)
    g = oracle.Geometry(64, 24, 91, extent=1.3, angles=tuple(np.concatenate([th, th + np.pi])))
    sino = oracle.project(g, 1, synth.random_image(32, 4))
    np.testing.assert_allclose(sino[12:], sino[:12, ::-1], rtol=0, atol=1e-11)


@pytest.mark.parametrize("lvl", [0, 2])
def test_listed_angles_dot_product_and_matrix(lvl):
    g, _ = _listed(64, 92, 21 + lvl, n_angles=50, extent=0.8)
    nl = 64 >> lvl
    rng = np.random.default_rng(lvl)
    x = rng.standard_normal((nl, nl))
    y = rng.standard_normal((50, 92))
    lhs = np.vdot(oracle.project(g, lvl, x), y)
    rhs = np.vdot(x, oracle.backproject(g, lvl, y))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(x * x) * np.sum(y * y)) * 8
    gs, _ = _listed(8, 12, 31 + lvl, n_angles=6, extent=0.8)
    ns = 8 >> lvl
    A = oracle.dense_matrix(lambda e: oracle.project(gs, lvl, e), (ns, ns), 6 * 12)
    At = oracle.dense_matrix(lambda e: oracle.backproject(gs, lvl, e), (6, 12), ns * ns)
    assert np.array_equal(A, At.T) and np.count_nonzero(A) > 0


def test_square_line_integrals_match_the_projector():
    """The analytic chords of the Sec. 5 square insert (synth) against the
    Joseph projection of its raster: exact on axis-aligned interior rays,
    first-order close elsewhere."""
    errs = []
    for n in (64, 128, 256):
        g = oracle.Geometry(n, 12, 3 * n // 2)
        block = n // 8
        exact = synth.square_line_integrals(n, block, 3, 5, 12, 3 * n // 2)
        sino = oracle.project(g, 0, synth.square_insert(n, block, 3, 5))
        errs.append(np.abs(sino - exact).mean())
        mid = 3 * n // 4  # theta = 0, rays x = s through the square's columns
        np.testing.assert_allclose(sino[0, mid - 2:mid + 2], exact[0, mid - 2:mid + 2], rtol=0, atol=1e-12)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.4 * errs[0], errs
