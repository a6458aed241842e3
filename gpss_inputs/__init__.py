"""Seeded synthetic scene descriptions for Gaussian process statistical surfaces.

This package only *describes* inputs: primitive lists, grids of kernel variance
and mean offsets drawn from seeded generators, lights, cameras and sampler
settings.  It contains none of the rendering arithmetic (no density, extinction,
normal distribution or tracking code), so that both the CPU oracle and the GPU
library can consume the same inputs without sharing any of the method.
"""
from .scenes import (  # noqa: F401
    Scene,
    plane_scene,
    sphere_scene,
    mixed_scene,
    batch_scenes,
    offset_sphere_scene,
    config_scenes,
    grad_param_indices,
)
