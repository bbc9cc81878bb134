"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates* inputs: unit-cell meshes (icospheres, open tube
segments), lattice descriptors, incident-wave directions, point-source
positions and random vectors.  It holds none of the boundary element or fast
multipole arithmetic; the CPU oracle (``oracle/``) and the HIP library each
derive everything else (centroids, normals, quadrature, operators) on their
own from these raw inputs.
"""
from .meshes import icosphere, tube_segment, mesh_is_closed
from .configs import (Lattice, Workload, config_tiny, config_grid16, config_grid16_ground, config_batched_grids,
                      config_large_cell, config_barrier_r4b, config_barrier_ground, barrier_receivers, serving_stream, SOUND_SPEED, DENSITY)
from .rng import unit_directions, random_complex

__all__ = ["icosphere", "tube_segment", "mesh_is_closed", "Lattice", "Workload",
           "config_tiny", "config_grid16", "config_grid16_ground", "config_batched_grids", "config_large_cell", "config_barrier_r4b", "config_barrier_ground", "barrier_receivers",
           "serving_stream", "unit_directions", "random_complex", "SOUND_SPEED", "DENSITY"]
