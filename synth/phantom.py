"""Seeded phantoms and measurement data for 2-D parallel-beam CT.

Geometry conventions (shared by every consumer, stated once here):

* The image domain is the square [-E, E]^2 with E = 1 unless a generator is
  given another extent.  An N x N image has
  pixel size h = 2E/N; pixel (i, j) is row i, column j, with centre
  x_j = -E + (j + 1/2) h and y_i = -E + (i + 1/2) h, stored row-major.
* Projection angle a of n_angles is theta_a = a*pi/n_angles (uniform over
  [0, pi), as in the paper's parallel-beam experiments, Sec. 4.1), unless an
  explicit list of angles is used (angles_random draws one).
* Detector bin b of n_det has centre s_b = (b - (n_det-1)/2) * ds + s0 with
  ds = the full-resolution pixel size 2E/N and s0 = 0.
* A ray is the line {x cos(theta) + y sin(theta) = s}.

The phantom family (random ellipses) stands in for the XCAT and AAPM images
of the paper's Sec. 4, which are not reproduced here.  The measured data are
the *analytic* line integrals of the ellipses (not a discrete projector, so
no inverse crime), passed through Poisson counting noise and the log
transform, as in the paper's noisy CT simulations (Sec. 4.1-4.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

EXTENT = 1.0


@dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    a: float  # semi-axis along the rotated x direction
    b: float  # semi-axis along the rotated y direction
    phi: float  # rotation angle
    value: float  # additive intensity


def angles_uniform(n_angles: int) -> np.ndarray:
    return np.arange(n_angles, dtype=np.float64) * np.pi / n_angles


def angles_random(n_angles: int, seed: int, lo: float = 0.0, hi: float = 2.0 * np.pi) -> np.ndarray:
    """n_angles angles drawn uniformly from [lo, hi), in draw order."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n_angles)


def detector_centres(n: int, n_det: int, det_offset: float = 0.0, extent: float = EXTENT) -> np.ndarray:
    ds = 2.0 * extent / n
    return (np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0) * ds + det_offset


def pixel_centres(n: int, extent: float = EXTENT) -> np.ndarray:
    h = 2.0 * extent / n
    return -extent + (np.arange(n, dtype=np.float64) + 0.5) * h


def random_ellipses(seed: int, n_ellipses: int = 8) -> list[Ellipse]:
    """Random-ellipse phantom: centres uniform in the disk of radius 0.45,
    semi-axes U[0.08, 0.45], rotation U[0, pi), intensity U[0, 1]; an
    ellipse is redrawn until it lies inside the disk of radius 0.95."""
    rng = np.random.default_rng(seed)
    out: list[Ellipse] = []
    while len(out) < n_ellipses:
        rad = 0.45 * np.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * np.pi)
        cx, cy = rad * np.cos(ang), rad * np.sin(ang)
        a, b = rng.uniform(0.08, 0.45, size=2)
        phi = rng.uniform(0.0, np.pi)
        val = rng.uniform(0.0, 1.0)
        if np.hypot(cx, cy) + max(a, b) > 0.95:
            continue
        out.append(Ellipse(float(cx), float(cy), float(a), float(b), float(phi), float(val)))
    return out


def rasterize_ellipses(ells: list[Ellipse], n: int) -> np.ndarray:
    """Sample the additive ellipse phantom at the N x N pixel centres."""
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc, indexing="xy")  # X[i, j] = x_j, Y[i, j] = y_i
    img = np.zeros((n, n), dtype=np.float64)
    for e in ells:
        dx, dy = X - e.cx, Y - e.cy
        c, s = np.cos(e.phi), np.sin(e.phi)
        xr = c * dx + s * dy
        yr = -s * dx + c * dy
        img += e.value * ((xr / e.a) ** 2 + (yr / e.b) ** 2 <= 1.0)
    return img


def ellipse_line_integrals(ells: list[Ellipse], n: int, n_angles: int, n_det: int,
                           det_offset: float = 0.0) -> np.ndarray:
    """Exact line integrals of the ellipse phantom on the ray grid, [angle][bin].

    For an ellipse centred at c with semi-axes (a, b) rotated by phi, the
    chord along the ray at angle theta and offset s has length
    2ab sqrt(a_t^2 - s'^2)/a_t^2, where s' = s - (cx cos theta + cy sin theta)
    and a_t^2 = a^2 cos^2(theta-phi) + b^2 sin^2(theta-phi)."""
    th = angles_uniform(n_angles)[:, None]
    s = detector_centres(n, n_det, det_offset)[None, :]
    out = np.zeros((n_angles, n_det), dtype=np.float64)
    for e in ells:
        sp = s - (e.cx * np.cos(th) + e.cy * np.sin(th))
        at2 = (e.a * np.cos(th - e.phi)) ** 2 + (e.b * np.sin(th - e.phi)) ** 2
        inside = sp * sp < at2
        chord = np.where(inside, 2.0 * e.a * e.b * np.sqrt(np.maximum(at2 - sp * sp, 0.0)) / at2, 0.0)
        out += e.value * chord
    return out


def fan_ray_points(n: int, n_views: int, n_det: int, src_dist: float, det_dist: float, ds: float = 0.0,
                   det_offset: float = 0.0, betas=None, extent: float = EXTENT):
    """Source and detector points of every ray of a flat-detector fan beam,
    each [view, bin, xy]: view a has its source at D (cos b, sin b),
    b = 2 pi a / n_views (or the listed angle), and bin k sits at
    t_k = (k - (n_det-1)/2) ds + det_offset along (-sin b, cos b) on the
    detector line through -det_dist (cos b, sin b).  ds <= 0 selects the
    pixel size magnified onto the detector, 2E/n (D + det_dist)/D."""
    if ds <= 0:
        ds = 2.0 * extent / n * (src_dist + det_dist) / src_dist
    beta = 2 * np.pi * np.arange(n_views) / n_views if betas is None else np.asarray(betas, dtype=np.float64)
    t = (np.arange(n_det) - (n_det - 1) / 2.0) * ds + det_offset
    ec = np.stack([np.cos(beta), np.sin(beta)], -1)[:, None, :]
    et = np.stack([-np.sin(beta), np.cos(beta)], -1)[:, None, :]
    src = np.broadcast_to(src_dist * ec, (n_views, n_det, 2))
    det = -det_dist * ec + t[None, :, None] * et
    return src, det


def ellipse_integrals_through(ells: list[Ellipse], p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Exact integrals of the ellipse phantom along the lines through points
    p and q ([..., 2] each): on the line X = p + t u (u the unit direction)
    an ellipse occupies the t between the roots of its quadratic
    ((X - c) rotated by -phi, scaled by 1/a and 1/b, of unit norm)."""
    d = q - p
    u = d / np.linalg.norm(d, axis=-1, keepdims=True)
    out = np.zeros(p.shape[:-1], dtype=np.float64)
    for e in ells:
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        rx = p[..., 0] - e.cx
        ry = p[..., 1] - e.cy
        # coordinates in the ellipse frame, scaled to the unit circle
        px = (cp * rx + sp * ry) / e.a
        py = (-sp * rx + cp * ry) / e.b
        ux = (cp * u[..., 0] + sp * u[..., 1]) / e.a
        uy = (-sp * u[..., 0] + cp * u[..., 1]) / e.b
        A = ux * ux + uy * uy
        B = 2.0 * (px * ux + py * uy)
        C = px * px + py * py - 1.0
        disc = B * B - 4.0 * A * C
        out += e.value * np.where(disc > 0, np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)
    return out


def fan_ct_problem(n: int, n_views: int, n_det: int, src_dist: float, det_dist: float, i0: float,
                   phantom_seed: int, noise_seed: int, n_ellipses: int = 8):
    """(x_true, b) on the flat-detector fan beam (default bin spacing):
    rasterised phantom and noisy post-log data from the exact integrals."""
    ells = random_ellipses(phantom_seed, n_ellipses)
    x_true = rasterize_ellipses(ells, n)
    src, det = fan_ray_points(n, n_views, n_det, src_dist, det_dist)
    b = poisson_log_data(ellipse_integrals_through(ells, src, det), i0, noise_seed)
    return x_true, b


def poisson_log_data(line_integrals: np.ndarray, i0: float, seed: int) -> np.ndarray:
    """Counts n ~ Poisson(I0 exp(-p)); data b = -ln(max(n, 1)/I0)."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(i0 * np.exp(-line_integrals))
    return -np.log(np.maximum(counts, 1).astype(np.float64) / i0)


def ct_problem(n: int, n_angles: int, n_det: int, i0: float, phantom_seed: int,
               noise_seed: int, n_ellipses: int = 8):
    """(x_true, b): rasterised phantom and noisy post-log data, float64."""
    ells = random_ellipses(phantom_seed, n_ellipses)
    x_true = rasterize_ellipses(ells, n)
    p = ellipse_line_integrals(ells, n, n_angles, n_det)
    b = poisson_log_data(p, i0, noise_seed)
    return x_true, b


def disk_image(n: int, rho: float, cx: float = 0.0, cy: float = 0.0, extent: float = EXTENT) -> np.ndarray:
    """Unit disk of radius rho centred at (cx, cy), sampled at pixel centres."""
    xc = pixel_centres(n, extent)
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    return ((X - cx) ** 2 + (Y - cy) ** 2 <= rho * rho).astype(np.float64)


def square_insert(n: int, block: int, lo: int, hi: int, value: float = 1.0) -> np.ndarray:
    """Square insert whose edges lie on the grid of block x block cells
    (the paper's Sec. 5 test image): pixels with lo*block <= i, j < hi*block."""
    img = np.zeros((n, n), dtype=np.float64)
    img[lo * block:hi * block, lo * block:hi * block] = value
    return img


def square_line_integrals(n: int, block: int, lo: int, hi: int, n_angles: int, n_det: int,
                          value: float = 1.0) -> np.ndarray:
    """Exact line integrals of square_insert(n, block, lo, hi, value) on the
    ray grid, [angle][bin]: value times the length of the ray's chord through
    the square [x0, x1] x [y0, y1] (slab clipping of the line
    {s (cos, sin) + t (-sin, cos)})."""
    h = 2.0 * EXTENT / n
    x0, x1 = -EXTENT + lo * block * h, -EXTENT + hi * block * h  # rows and columns share the bounds
    th = angles_uniform(n_angles)[:, None]
    s = detector_centres(n, n_det)[None, :]
    c, sn = np.cos(th), np.sin(th)
    px, py, dx, dy = s * c, s * sn, -sn, c  # point on the ray and its direction
    tmin = np.full(np.broadcast(px, dx).shape, -np.inf)
    tmax = np.full_like(tmin, np.inf)
    for p0, d in ((px, dx), (py, dy)):
        d = np.broadcast_to(d, tmin.shape)
        p0 = np.broadcast_to(p0, tmin.shape)
        par = np.abs(d) < 1e-300
        with np.errstate(divide="ignore", invalid="ignore"):
            t1, t2 = (x0 - p0) / d, (x1 - p0) / d
        lo_t, hi_t = np.minimum(t1, t2), np.maximum(t1, t2)
        inside = (p0 >= x0) & (p0 <= x1)
        tmin = np.where(par, np.where(inside, tmin, np.inf), np.maximum(tmin, lo_t))
        tmax = np.where(par, np.where(inside, tmax, -np.inf), np.minimum(tmax, hi_t))
    return value * np.maximum(tmax - tmin, 0.0)


def affine_image(n: int, alpha: float, beta: float, gamma: float, extent: float = EXTENT) -> np.ndarray:
    """f(x, y) = alpha x + beta y + gamma at the pixel centres."""
    xc = pixel_centres(n, extent)
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    return alpha * X + beta * Y + gamma


def random_image(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))


def random_sinogram(n_angles: int, n_det: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n_angles, n_det))
