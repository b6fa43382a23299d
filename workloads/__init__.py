"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This package holds no arithmetic of the summation method itself: it draws
points, weights and direction sets (the random quantities the method takes as
inputs) and picks the kernel width by the median rule.  Both the FP64 oracle
and the GPU path receive these arrays as plain inputs; neither imports the
other.
"""
from .points import (unit_ball, gaussian_mixture, image_like, mmd_particles,
                     median_rule_sigma)
from .directions import (iid_directions, sobol_directions, orthogonal_directions,
                         distance_qmc_directions, random_rotation, directions)
from .configs import CONFIGS, make_config

__all__ = [
    "unit_ball", "gaussian_mixture", "image_like", "mmd_particles",
    "median_rule_sigma", "iid_directions", "sobol_directions",
    "orthogonal_directions", "distance_qmc_directions", "random_rotation",
    "directions", "CONFIGS", "make_config",
]
