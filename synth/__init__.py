"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package generates problem instances only: closed triangulated surfaces
(icosphere, box/cube, thin film), a seeded smooth magnetisation field, and the
surface density sampled at the triangle quadrature points. It contains none of
the single-layer-potential arithmetic (no scaling to the torus, no kernel
coefficients, no window, no transforms); both the HIP library and the oracle
do that work independently from these arrays.
"""
from .meshes import (icosphere, box_surface, cube, cube_volume_nodes, box_tets, cube_tets, ball_tets,
                     thin_film, mesh_summary)
from .fields import RandomSmoothMagnetisation, uniform_magnetisation
from .density import quadrature_sample_points, density_from_magnetisation
from .workloads import Workload, make_workload, WORKLOADS

__all__ = [
    "cube_volume_nodes", "box_tets", "cube_tets", "ball_tets",
    "icosphere", "box_surface", "cube", "thin_film", "mesh_summary",
    "RandomSmoothMagnetisation", "uniform_magnetisation",
    "quadrature_sample_points", "density_from_magnetisation",
    "Workload", "make_workload", "WORKLOADS",
]
