"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Nothing in this package computes any part of the method: it only places
spheres, draws radii and draws forces, so that the CPU oracle and the GPU
library see identical inputs.
"""
from .spheres import (  # noqa: F401
    A_FCC,
    fcc_ball_sites,
    sphere_cluster,
    batched_sizes,
    batched_instance,
    dynamics_noise,
)
