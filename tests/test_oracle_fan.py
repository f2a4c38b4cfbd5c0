"""Pins of the oracle's fan-beam projector pair (CPU only).

The fan beam (source at distance D from the centre on a circle, flat detector
at distance Dd beyond it, rays from the source to the bin centres) is the
divergent-beam case of the paper's line-integral operator (Sec. 4.1; the
outlook of Sec. 6 names other geometries).  What pins it, each check
computed here without the oracle's own line construction:
  * closed-form chords of an off-centre disk, with each ray built as the
    line through the source point and its detector point (a cross product,
    not the oracle's normal vector), converging at first order;
  * exactness on affine images (Joseph sums are exact for linear integrands
    whose taps stay inside the image), on every level;
  * the limit D -> infinity (Dd = 0) is the parallel beam with angles
    beta + pi/2 and the same bins;
  * the dot-product test and explicit matrices: the transpose is the forward
    matrix transposed, bit for bit;
  * Alg. 1 on a fan geometry converges to the dense Tikhonov minimiser;
  * the fan workload's analytic ellipse data (synth) against the oracle's
    projection of the rasterised phantom, first order, with synth's
    two-point chord checked against its parallel closed form first.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth


def _rays(n_views, n_det, D, Dd, ds, s0=0.0, betas=None):
    """Source and detector points of every ray, [view, bin, xy]."""
    beta = 2 * np.pi * np.arange(n_views) / n_views if betas is None else np.asarray(betas)
    t = (np.arange(n_det) - (n_det - 1) / 2.0) * ds + s0
    ec = np.stack([np.cos(beta), np.sin(beta)], -1)[:, None, :]
    et = np.stack([-np.sin(beta), np.cos(beta)], -1)[:, None, :]
    src = D * ec + 0 * t[None, :, None]
    det = -Dd * ec + t[None, :, None] * et
    return src, det


def _chords(src, det, rho, cx, cy):
    d = det - src
    c = np.array([cx, cy])
    cr = d[..., 0] * (c[1] - src[..., 1]) - d[..., 1] * (c[0] - src[..., 0])
    dist = np.abs(cr) / np.linalg.norm(d, axis=-1)
    return 2.0 * np.sqrt(np.maximum(rho * rho - dist * dist, 0.0)), dist


def test_fan_disk_chords_converge_first_order():
    E, D, Dd = 1.3, 4.0, 2.5
    cx, cy, rho = 0.21 * E, -0.13 * E, 0.5 * E
    means = []
    for n in (64, 128, 256, 512):
        nd = 3 * n // 2
        g = oracle.Geometry(n, 24, nd, extent=E, src_dist=D * E, det_dist=Dd * E)
        sino = oracle.project(g, 0, synth.disk_image(n, rho, cx, cy, extent=E))
        src, det = _rays(24, nd, D * E, Dd * E, g.spacing)
        exact, dist = _chords(src, det, rho, cx, cy)
        err = np.abs(sino - exact)
        d = det - src
        step = (2.0 * E / n) * np.linalg.norm(d, axis=-1) / np.maximum(np.abs(d[..., 0]), np.abs(d[..., 1]))
        assert (err / step)[dist <= 0.9 * rho].max() < 2.0, n
        means.append(err.mean())
    ratios = np.array(means[1:]) / np.array(means[:-1])
    assert ratios.max() < 0.65, ratios
    assert means[-1] / means[0] < 0.2


@pytest.mark.parametrize("lvl", [0, 1, 2])
def test_fan_affine_images_are_exact(lvl):
    n, nv, nd, E, D, Dd = 64, 40, 96, 1.7, 6.0, 3.0
    g = oracle.Geometry(n, nv, nd, extent=E, src_dist=D, det_dist=Dd, s0=0.05)
    alpha, beta, gamma = 0.7, -0.45, 0.3
    nl = n >> lvl
    h = 2.0 * E / nl
    sino = oracle.project(g, lvl, synth.affine_image(nl, alpha, beta, gamma, extent=E))
    src, det = _rays(nv, nd, D, Dd, g.spacing, 0.05)
    c0 = -E + 0.5 * h
    ends = np.array([c0, -c0])
    checked = 0
    for a in range(nv):
        for b in range(nd):
            p, q = src[a, b], det[a, b]
            dx, dy = q - p
            if abs(dy) >= abs(dx):  # steep: crosses every row once (row stepping)
                xs = p[0] + (ends - p[1]) * dx / dy  # x at the first and last row centres
                u = (xs - c0) / h
                x0 = p[0] - p[1] * dx / dy            # x where the line crosses y = 0
                expect = 2.0 * E * np.hypot(dx, dy) / abs(dy) * (alpha * x0 + gamma)
            else:
                ys = p[1] + (ends - p[0]) * dy / dx
                u = (ys - c0) / h
                y0 = p[1] - p[0] * dy / dx
                expect = 2.0 * E * np.hypot(dx, dy) / abs(dx) * (beta * y0 + gamma)
            if u.min() >= 0.0 and u.max() <= nl - 1:
                assert abs(sino[a, b] - expect) <= 1e-11 * max(1.0, abs(expect)), (a, b)
                checked += 1
    assert checked > nv * 10


def test_fan_tends_to_parallel_beam():
    n, nv, nd = 64, 30, 92
    betas = synth.angles_random(nv, 3, 0.0, 2 * np.pi)
    ds = 2.0 / n
    fan = oracle.Geometry(n, nv, nd, ds=ds, s0=0.01, src_dist=1e8, det_dist=0.0, angles=tuple(betas))
    par = oracle.Geometry(n, nv, nd, ds=ds, s0=0.01, angles=tuple(betas + np.pi / 2))
    z = synth.random_image(n, 5)
    y = synth.random_sinogram(nv, nd, 6)
    for lvl in (0, 2):
        zl = z[:n >> lvl, :n >> lvl]
        np.testing.assert_allclose(oracle.project(fan, lvl, zl), oracle.project(par, lvl, zl), rtol=0, atol=1e-6)
        np.testing.assert_allclose(oracle.backproject(fan, lvl, y), oracle.backproject(par, lvl, y), rtol=0,
                                   atol=1e-6)
    # a short source distance is far from it
    near = oracle.Geometry(n, nv, nd, ds=ds, s0=0.01, src_dist=3.0, det_dist=0.0, angles=tuple(betas))
    assert np.abs(oracle.project(near, 0, z) - oracle.project(par, 0, z)).max() > 1e-2


@pytest.mark.parametrize("lvl", [0, 1, 2])
def test_fan_dot_product_and_matrix(lvl):
    g = oracle.Geometry(64, 50, 80, extent=0.9, src_dist=3.1, det_dist=1.7, s0=-0.02)
    nl = 64 >> lvl
    rng = np.random.default_rng(lvl)
    x = rng.standard_normal((nl, nl))
    y = rng.standard_normal((50, 80))
    lhs = np.vdot(oracle.project(g, lvl, x), y)
    rhs = np.vdot(x, oracle.backproject(g, lvl, y))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(x * x) * np.sum(y * y)) * 8
    gs = oracle.Geometry(8, 6, 14, extent=0.9, src_dist=2.9, det_dist=1.1)
    ns = 8 >> lvl
    A = oracle.dense_matrix(lambda e: oracle.project(gs, lvl, e), (ns, ns), 6 * 14)
    At = oracle.dense_matrix(lambda e: oracle.backproject(gs, lvl, e), (6, 14), ns * ns)
    assert np.array_equal(A, At.T) and np.count_nonzero(A) > 0


def test_fan_alg1_converges_to_dense_minimiser():
    g = oracle.Geometry(16, 30, 28, src_dist=3.0, det_dist=2.0)
    lv = oracle.Levels([0, 1, 2], [0.4, 0.3, 0.3], oracle.MODE_UNBIASED)
    _, b = synth.ct_problem(16, 30, 28, 1e4, 1040, 2040)
    lam = 0.1
    K = oracle.dense_matrix(lambda e: oracle.project(g, 0, e), (16, 16), 30 * 28)
    xs = sl.solve(K.T @ K + lam * np.eye(256), K.T @ b.ravel(), assume_a="pos").reshape(16, 16)
    st = None
    errs = []
    for _ in range(6):
        st = oracle.imask_run(g, lv, oracle.Reg(lam=lam), 0.02, 42, 0, b, 1500, st)
        errs.append(np.linalg.norm(st.x - xs) / np.linalg.norm(xs))
    assert errs[-1] < 1e-8, errs
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))


def test_ellipse_integrals_through_points_reproduce_the_parallel_closed_form():
    """synth's chord through two points equals its parallel-beam chord
    formula on parallel rays (two independent closed forms)."""
    ells = synth.random_ellipses(1000, 8)
    n, na, nd = 64, 30, 96
    th = synth.angles_uniform(na)[:, None] + 0 * np.zeros(nd)[None, :]
    s = synth.detector_centres(n, nd)[None, :] + 0 * th
    p = np.stack([s * np.cos(th), s * np.sin(th)], -1)
    q = p + np.stack([-np.sin(th), np.cos(th)], -1)
    got = synth.ellipse_integrals_through(ells, p, q)
    np.testing.assert_allclose(got, synth.ellipse_line_integrals(ells, n, na, nd), rtol=0, atol=1e-12)


def test_fan_ellipse_data_matches_the_oracle_projector():
    """The fan workload's analytic data against the oracle's Joseph projection
    of the rasterised phantom: first-order convergence (pins the fan ray
    construction of synth and of the oracle against each other)."""
    errs = []
    for n in (64, 128, 256):
        ells = synth.random_ellipses(1000, 8)
        x = synth.rasterize_ellipses(ells, n)
        src, det = synth.fan_ray_points(n, 24, 3 * n // 2, 4.0, 2.0)
        exact = synth.ellipse_integrals_through(ells, src, det)
        g = oracle.Geometry(n, 24, 3 * n // 2, src_dist=4.0, det_dist=2.0)
        errs.append(np.linalg.norm(oracle.project(g, 0, x) - exact) / np.linalg.norm(exact))
    assert errs[0] < 0.03 and errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs
