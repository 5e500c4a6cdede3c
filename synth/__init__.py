"""Seeded synthetic inputs for the OS-LALM CT workloads.

This package only *generates inputs*: scanner geometries, random
ellipse/ellipsoid phantoms, their analytic line integrals, Poisson counts and
evaluation masks.  It contains none of the reconstruction method's arithmetic
(no system matrix, no gradients, no updates); both the FP64 oracle and the
HIP library consume what it produces, and neither is imported here.
"""
from .configs import CONFIGS, get_config, geometry_of, HU_PER_MU, MU_WATER
from .phantom import (make_phantom, ray_sources_directions, analytic_sinogram,
                      noisy_data, pixelize, roi_mask, roi_radius, fov_radius,
                      make_problem_data)

__all__ = [
    "CONFIGS", "get_config", "geometry_of", "HU_PER_MU", "MU_WATER",
    "make_phantom", "ray_sources_directions", "analytic_sinogram",
    "noisy_data", "pixelize", "roi_mask", "roi_radius", "fov_radius", "make_problem_data",
]
