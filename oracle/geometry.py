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


def density_p1(nodes, tris, m_nodes, dphi1_dn=None):
    """Element-constant density g_j = (1/|S_j|) int_{S_j} m.n - dphi1/dn_j of the P1
    ansatz (Sec. 2): m is the affine nodal interpolant on each flat triangle, its
    normal component is projected onto constants by the integral mean, and the
    normal derivative of phi_1 is already constant per triangle. The integral is
    taken with the degree-2 rule of `quadrature`, exact for affine integrands.
    Returns g_k for the long index k = j + s*M (the same value for s = 0, 1, 2)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    m_nodes = np.asarray(m_nodes, dtype=np.float64)
    M = tris.shape[0]
    area, nrm = triangle_areas_normals(nodes, tris)
    integral = np.zeros(M)
    for s in range(3):
        m_at_y = (_B[s, 0] * m_nodes[tris[:, 0]] + _B[s, 1] * m_nodes[tris[:, 1]]
                  + _B[s, 2] * m_nodes[tris[:, 2]])
        integral += area / 3.0 * (m_at_y * nrm).sum(axis=1)
    g = integral / area
    if dphi1_dn is not None:
        g = g - np.asarray(dphi1_dn, dtype=np.float64)
    return np.tile(g, 3)
