"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws meshes and random data.  It holds none of the
multigrid arithmetic (no Laplacian, mass matrix, prolongation, coloring or
solver step): each side computes those itself from what is generated here.
"""
from .meshes import (icosphere_subdiv, icosphere_freq, torus_grid, disc_grid,
                     mean_edge_length, edges_of)
from .workloads import (workload_c1, workload_c2, workload_c3, workload_c4,
                        workload_c5_mesh, workload_c5_frame, small_icosphere,
                        flat_disc)

__all__ = [
    "icosphere_subdiv", "icosphere_freq", "torus_grid", "disc_grid",
    "mean_edge_length", "edges_of", "workload_c1", "workload_c2", "workload_c3",
    "workload_c4", "workload_c5_mesh", "workload_c5_frame", "small_icosphere",
    "flat_disc",
]
