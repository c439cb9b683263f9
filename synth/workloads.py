"""Named, seeded problem instances shaped like the paper's workloads.

Each workload is a closed surface mesh, a density sampled at the quadrature
points, the oversampled FFT grid, the window cut-off and the specification of
the exponential-sum approximation of 1/r (step h, validity interval
[r_lo, r_hi], lower-tail tolerance). The exponential sum itself is computed by
whoever consumes the workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import icosphere, cube, thin_film
from .fields import RandomSmoothMagnetisation, uniform_magnetisation
from .density import density_from_magnetisation


@dataclass
class Workload:
    name: str
    nodes: np.ndarray
    tris: np.ndarray
    dens: np.ndarray
    grid: tuple
    m: int
    alpha: int = 2
    eta2: float = 37.0
    es_h: float = 0.2
    es_r_lo: float = 0.0
    es_r_hi: float = 0.0
    es_tol: float = 1e-12
    meta: dict = field(default_factory=dict)

    @property
    def n_src(self) -> int:
        return 3 * int(self.tris.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])


def expsum_interval(nodes):
    """[r_lo, r_hi] for the exponential sum: r_hi = bounding-box diagonal,
    r_lo = 1e-3 * r_hi (physical units)."""
    ext = nodes.max(axis=0) - nodes.min(axis=0)
    r_hi = float(np.linalg.norm(ext))
    return 1e-3 * r_hi, r_hi


def _finish(name, nodes, tris, dens, grid, m, **kw):
    r_lo, r_hi = expsum_interval(nodes)
    return Workload(name=name, nodes=nodes, tris=tris, dens=dens,
                    grid=tuple(int(g) for g in grid), m=int(m),
                    es_r_lo=r_lo, es_r_hi=r_hi, **kw)


def sphere_uniform(level=3, grid=64, m=8, radius=1.0):
    nodes, tris = icosphere(level, radius)
    dens = density_from_magnetisation(nodes, tris, uniform_magnetisation())
    return _finish(f"sphere_l{level}", nodes, tris, dens, (grid,) * 3, m,
                   meta={"magnetisation": "uniform (0,0,1)"})


def sphere_random(level, seed, grid, m):
    nodes, tris = icosphere(level, 1.0)
    mf = RandomSmoothMagnetisation(seed, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    return _finish(f"sphere_l{level}_s{seed}", nodes, tris, dens, (grid,) * 3, m,
                   meta={"seed": seed})


def cube_random(cells=64, seed=2, grid=128, m=8):
    nodes, tris = cube(cells)
    mf = RandomSmoothMagnetisation(seed, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    return _finish(f"cube{cells}_s{seed}", nodes, tris, dens, (grid,) * 3, m,
                   meta={"seed": seed})


def film_random(cells_xy=512, cells_z=10, seed=3, grid=(1024, 1024, 64), m=4):
    nodes, tris = thin_film(cells_xy, cells_z)
    mf = RandomSmoothMagnetisation(seed, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    return _finish(f"film{cells_xy}_s{seed}", nodes, tris, dens, grid, m,
                   meta={"seed": seed})


WORKLOADS = {
    # icosphere L3 (1280 tris, 642 nodes), uniform m = (0,0,1), grid 64^3
    "sphere_l3": lambda m=8: sphere_uniform(3, 64, m),
    # unit cube 64x64 cells per face (49152 tris, 24578 nodes), seed 2, grid 128^3
    "cube64": lambda m=8: cube_random(64, 2, 128, m),
    # film 1 x 1 x 0.02 (1089536 tris, 544770 nodes), seed 3, grid 1024x1024x64
    "film512": lambda m=4: film_random(512, 10, 3, (1024, 1024, 64), m),
}


def make_workload(name: str, m=None) -> Workload:
    f = WORKLOADS[name]
    return f() if m is None else f(m)
