"""Seeded synthetic inputs for the matrix-pencil Prony method.

This package draws random numbers only: nodes t_j, coefficients c_j, noise
arrays, the random unit vector mu and random starting blocks. It holds none of
the method's arithmetic (no samples, no Toeplitz matrices, no products), so
both the CPU oracle and the GPU path can consume the same draws.
"""
from .generate import (  # noqa: F401
    MASTER_SEED,
    Instance,
    config_instances,
    draw_instance,
    paper_efficiency_inputs,
    paper_relative_noise,
    random_unit_vector,
    random_orthonormal,
    torus_distance,
)
