"""Seeded synthetic voxel images shared by the oracle, the tests and the bench.

This package holds only input generation (solid/fluid masks and per-voxel
force fields).  It contains none of the lattice-Boltzmann arithmetic, so both
the FP64 oracle and the HIP path can consume its output without sharing any
method code.
"""
from .geometry import (  # noqa: F401
    sphere,
    slit,
    duct,
    pipe,
    triangle_channel,
    sphere_pack,
    gaussian_random_field,
    percolating_x,
    crop,
    random_mask,
    porosity,
    workload,
    WORKLOADS,
)
