"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package only draws phantoms and evaluates their analytic parallel-beam
Radon transforms (data synthesis). It holds none of the backprojection
arithmetic of the method under test.
"""
from .phantoms import (  # noqa: F401
    Geometry,
    Ellipse,
    Gaussian,
    random_ellipses,
    head_phantom,
    ellipse_sinogram,
    ellipse_image,
    gaussian_sinogram,
    gaussian_image,
    add_gaussian_noise,
    ellipsoid_volume_params,
    ellipsoid_slice_ellipses,
    poisson_like_noise,
    config1_sinogram,
    batch_sinograms,
)
