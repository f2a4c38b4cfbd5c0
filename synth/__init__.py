"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package produces phantoms, analytic sinograms, Poisson noise and random
test vectors.  It holds none of the reconstruction method's arithmetic (no
projector, no resampling operator, no iteration): both the oracle and the
GPU library consume what it makes, and neither one's code lives here.
"""
from .phantom import (  # noqa: F401
    Ellipse,
    random_ellipses,
    rasterize_ellipses,
    ellipse_line_integrals,
    poisson_log_data,
    detector_centres,
    angles_uniform,
    angles_random,
    pixel_centres,
    disk_image,
    square_insert,
    square_line_integrals,
    affine_image,
    random_image,
    random_sinogram,
    ct_problem,
    fan_ray_points,
    ellipse_integrals_through,
    fan_ct_problem,
)
