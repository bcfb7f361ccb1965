"""Seeded synthetic particle generators shared by the tests and the benchmark.

This package holds no compressor arithmetic: it only draws particle
positions with the shapes and value distributions of the paper's workloads
(cosmology-, fluid- and fusion-shaped sets, Table 2 of the paper), since the paper's
datasets are not available.
"""
from .generators import (  # noqa: F401
    uniform_cube,
    cosmology,
    fluid,
    fluid_lattice_dims,
    poincare,
    batch_plan,
    batch_set,
    batch_sets,
    served_requests,
    request_pool,
    poisson_arrivals,
    sha256_of,
)
