"""Quadrature on flat triangles and the scaling of the body into the torus.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

# Degree-2 interior rule on a triangle: three points, equal weights |S|/3.
# Point s has barycentric coordinate 2/3 on vertex s and 1/6 on the others.
_B = np.array([[4.0, 1.0, 1.0], [1.0, 4.0, 1.0], [1.0, 1.0, 4.0]]) / 6.0


def triangle_areas_normals(nodes, tris):
    """Area |S_j| and unit normal of every flat triangle S_j (eq. triangle:
    y = y0 + xi1 (y1 - y0) + xi2 (y2 - y0))."""
    y0 = nodes[tris[:, 0]]
    cr = np.cross(nodes[tris[:, 1]] - y0, nodes[tris[:, 2]] - y0)
    two_area = np.sqrt((cr * cr).sum(axis=1))
    return 0.5 * two_area, cr / two_area[:, None]


def quadrature(nodes, tris):
    """Quadrature points y_k and weights w_k for the surface integral.

    Long index k = j + s*M (triangle j = 0..M-1, point s = 0..2), as in the
    discrete sum of eq. (naive_gridding). Returns y [3M, 3], w [3M]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    M = tris.shape[0]
    area, _ = triangle_areas_normals(nodes, tris)
    ys = []
    for s in range(3):
        ys.append(_B[s, 0] * nodes[tris[:, 0]] + _B[s, 1] * nodes[tris[:, 1]]
                  + _B[s, 2] * nodes[tris[:, 2]])
    y = np.concatenate(ys, axis=0)
    w = np.tile(area / 3.0, 3)
    assert y.shape == (3 * M, 3)
    return y, w


def scaling(nodes, grid):
    """Centre c and per-axis factors s_q mapping the body into (-0.2, 0.2)^3.

    The paper scales the body into the box (-0.2, 0.2)^3 inside the torus
    T = [-1/2, 1/2)^3 (Sec. 4). Reading used here: c is the bounding-box
    centre and s_q N_q is the same on every axis (equal physical grid spacing),
    chosen as large as possible with every scaled coordinate in [-0.2, 0.2]:
    s_q = K / N_q, K = min_q 0.4 N_q / extent_q."""
    nodes = np.asarray(nodes, dtype=np.float64)
    lo, hi = nodes.min(axis=0), nodes.max(axis=0)
    c = 0.5 * (lo + hi)
    ext = hi - lo
    N = np.asarray(grid, dtype=np.float64)
    ratios = np.where(ext > 0, 0.4 * N / np.where(ext > 0, ext, 1.0), np.inf)
    K = ratios.min()
    return c, K / N


def to_torus(x, c, s):
    """x~ = S (x - c)."""
    return (np.asarray(x, dtype=np.float64) - c) * s
