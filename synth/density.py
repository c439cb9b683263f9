"""Surface density g = m . n sampled at the triangle quadrature points.

The density is the input of the single-layer potential (the Dirichlet-part
normal derivative is taken as zero here, so g = m . n). It is sampled at the
degree-2 interior three-point rule of every flat triangle, in the long index
order k = j + s*M (triangle j, point s): the same points at which the library
and the oracle place their sources. Point s carries barycentric weight 2/3 on
vertex s and 1/6 on the other two.
"""
from __future__ import annotations

import numpy as np

_BARY = np.array([[2 / 3, 1 / 6, 1 / 6],
                  [1 / 6, 2 / 3, 1 / 6],
                  [1 / 6, 1 / 6, 2 / 3]], dtype=np.float64)


def quadrature_sample_points(nodes, tris):
    """Sample points [3M, 3] in long index order and unit outward normals [M, 3]."""
    p = nodes[tris]                                   # [M, 3 vertices, 3]
    pts = np.einsum("sv,mvd->smd", _BARY, p).reshape(-1, 3)
    nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


def density_from_magnetisation(nodes, tris, mfield):
    """g_k = m(y_k) . n_j for k = j + s*M (float64 [3M])."""
    pts, nrm = quadrature_sample_points(nodes, tris)
    M = tris.shape[0]
    mv = mfield(pts)
    return np.einsum("kd,kd->k", mv, np.tile(nrm, (3, 1))).astype(np.float64)
