"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random numbers and lays out particle configurations. It holds
none of the method's arithmetic (no kernel, no tree, no partition, no ACA).
"""
from .gen import (  # noqa: F401
    Rng,
    cube_side,
    drop_radius,
    rsa_cube,
    lattice_sphere,
    lattice_cube,
    filament_chains,
    filament_suspension,
    batch_workload,
    normal_forces,
    gravity_forces,
    mlp_weights,
    sample_rows,
    batch_systems,
    workload,
    WORKLOADS,
)
