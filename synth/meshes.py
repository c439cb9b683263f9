"""Closed, outward-oriented triangle surface meshes (flat affine triangles).

Node arrays are float64 [N, 3]; triangle arrays are int32 [M, 3], 0-based,
counter-clockwise seen from outside (so the cross product of the two edge
vectors points outward).
"""
from __future__ import annotations

import numpy as np


def icosphere(level: int, radius: float = 1.0):
    """Icosahedron refined `level` times by edge midpoints, vertices projected
    onto the sphere of the given radius.  Counts: 20*4^L triangles,
    10*4^L + 2 vertices."""
    if level < 0:
        raise ValueError("level must be >= 0")
    p = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
             (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
             (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.asarray(x, dtype=np.float64) / np.linalg.norm(x) for x in verts]
    f = list(faces)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                c = v[a] + v[b]
                v.append(c / np.linalg.norm(c))
                idx = len(v) - 1
                cache[key] = idx
            return idx

        nf = []
        for (a, b, c) in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    nodes = np.array(v, dtype=np.float64) * float(radius)
    tris = np.array(f, dtype=np.int32)
    _orient_outward(nodes, tris, centre=np.zeros(3))
    return nodes, tris


def box_surface(extent, cells, centre=(0.0, 0.0, 0.0)):
    """Surface of the axis-aligned box of the given extent, centred at `centre`,
    with cells[q] structured cells along axis q. Every rectangular face cell is
    split into two triangles along its (i, j) -> (i+1, j+1) diagonal. Nodes are
    the lattice points on the box surface (shared by neighbouring faces)."""
    ex = np.asarray(extent, dtype=np.float64)
    cx, cy, cz = (int(c) for c in cells)
    if min(cx, cy, cz) < 1:
        raise ValueError("cells must be >= 1 along every axis")
    dims = (cx + 1, cy + 1, cz + 1)
    ii, jj, kk = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]),
                             np.arange(dims[2]), indexing="ij")
    on_surf = ((ii == 0) | (ii == cx) | (jj == 0) | (jj == cy) |
               (kk == 0) | (kk == cz))
    node_id = -np.ones(dims, dtype=np.int64)
    n_nodes = int(on_surf.sum())
    node_id[on_surf] = np.arange(n_nodes)
    lat = np.stack([ii[on_surf], jj[on_surf], kk[on_surf]], axis=1)
    nodes = (lat / np.array([cx, cy, cz], dtype=np.float64) - 0.5) * ex
    nodes = nodes + np.asarray(centre, dtype=np.float64)

    tris = []
    # Each face: fixed axis `a` at index 0 or max; the two free axes (u, v).
    for a in range(3):
        u, v = [q for q in range(3) if q != a]
        nu, nv = (cx, cy, cz)[u], (cx, cy, cz)[v]
        for side in (0, (cx, cy, cz)[a]):
            iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
            iu = iu.ravel()
            iv = iv.ravel()

            def nid(du, dv):
                idx = [None, None, None]
                idx[a] = np.full(iu.shape, side)
                idx[u] = iu + du
                idx[v] = iv + dv
                return node_id[idx[0], idx[1], idx[2]]

            p00, p10, p11, p01 = nid(0, 0), nid(1, 0), nid(1, 1), nid(0, 1)
            t1 = np.stack([p00, p10, p11], axis=1)
            t2 = np.stack([p00, p11, p01], axis=1)
            tris.append(np.concatenate([t1, t2], axis=0))
    tris = np.concatenate(tris, axis=0).astype(np.int32)
    _orient_outward(nodes, tris, centre=np.asarray(centre, dtype=np.float64))
    return nodes, tris


def cube(cells_per_edge: int):
    """Unit cube [-1/2, 1/2]^3, cells_per_edge^2 cells on every face."""
    c = int(cells_per_edge)
    return box_surface((1.0, 1.0, 1.0), (c, c, c))


def cube_volume_nodes(cells_per_edge: int):
    """Nodes of the structured tetrahedral mesh of the unit cube whose boundary
    triangulation is cube(cells_per_edge): the (c+1)^3 lattice points of
    [-1/2, 1/2]^3 (every lattice cell split into tetrahedra adds no node).
    Its boundary points are exactly the nodes of cube(c)."""
    c = int(cells_per_edge)
    t = np.linspace(-0.5, 0.5, c + 1)
    x, y, z = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def box_tets(extent, cells):
    """Structured tetrahedral mesh of the box of the given extent centred at 0:
    the lattice points (index (i (cy+1) + j)(cz+1) + k for lattice point
    (i, j, k)) and every lattice cell split into the six tetrahedra that share
    its diagonal from the lowest to the highest corner (one per order of the
    three axes). Each boundary face of a cell is then split along its
    (i, j) -> (i+1, j+1) diagonal, as in box_surface. Tetrahedra are positively
    oriented. Returns (nodes [(cx+1)(cy+1)(cz+1), 3], tets int32 [6 cx cy cz, 4])."""
    ex = np.asarray(extent, dtype=np.float64)
    cx, cy, cz = (int(c) for c in cells)
    axes = [np.linspace(-0.5 * ex[q], 0.5 * ex[q], n + 1) for q, n in enumerate((cx, cy, cz))]
    x, y, z = np.meshgrid(*axes, indexing="ij")
    nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    ii, jj, kk = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    tets = []
    for order in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        corner = base.copy()
        verts = [corner.copy()]
        for ax in order:
            corner[:, ax] += 1
            verts.append(corner.copy())
        ids = [(v[:, 0] * (cy + 1) + v[:, 1]) * (cz + 1) + v[:, 2] for v in verts]
        tets.append(np.stack(ids, axis=1))
    tets = np.concatenate(tets, axis=0).astype(np.int32)
    return nodes, _orient_tets(nodes, tets)


def cube_tets(cells_per_edge: int):
    """box_tets of the unit cube [-1/2, 1/2]^3 with c cells per edge: its nodes
    are cube_volume_nodes(c) in the same order and its boundary faces the
    triangles of cube(c)."""
    c = int(cells_per_edge)
    return box_tets((1.0, 1.0, 1.0), (c, c, c))


def ball_tets(cells_per_edge: int, radius: float = 1.0):
    """cube_tets(c) mapped onto the ball of the given radius by
    x -> 2 radius x |x|_inf / |x|_2 (the cube's boundary onto the sphere; the
    map is continuous and one-to-one, tetrahedra keep their orientation for the
    sizes used here)."""
    nodes, tets = cube_tets(cells_per_edge)
    r2 = np.linalg.norm(nodes, axis=1)
    rinf = np.abs(nodes).max(axis=1)
    fac = np.where(r2 > 0, 2.0 * radius * rinf / np.where(r2 > 0, r2, 1.0), 0.0)
    return nodes * fac[:, None], tets


def _orient_tets(nodes, tets):
    """Swap two vertices of every negatively oriented tetrahedron."""
    P = nodes[tets]
    vol = np.einsum("ij,ij->i", np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0])
    neg = vol < 0
    if np.any(neg):
        tets[neg] = tets[neg][:, [0, 2, 1, 3]]
    return tets


def thin_film(cells_xy: int = 512, cells_z: int = 10, thickness: float = 0.02):
    """Thin film 1 x 1 x thickness: cells_xy^2 cells on the large faces and
    cells_xy x cells_z cells on each side face."""
    return box_surface((1.0, 1.0, float(thickness)), (cells_xy, cells_xy, cells_z))


def _orient_outward(nodes, tris, centre):
    """Flip triangles whose normal points towards `centre` (convex bodies)."""
    p0 = nodes[tris[:, 0]]
    nrm = np.cross(nodes[tris[:, 1]] - p0, nodes[tris[:, 2]] - p0)
    cen = (p0 + nodes[tris[:, 1]] + nodes[tris[:, 2]]) / 3.0
    flip = np.einsum("ij,ij->i", nrm, cen - centre) < 0
    if np.any(flip):
        tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def mesh_summary(nodes, tris):
    """Counts and closedness facts used by the mesh tests."""
    edges = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    und = np.sort(edges, axis=1)
    uniq, counts = np.unique(und, axis=0, return_counts=True)
    return {
        "nodes": int(nodes.shape[0]),
        "tris": int(tris.shape[0]),
        "edges": int(uniq.shape[0]),
        "every_edge_shared_twice": bool(np.all(counts == 2)),
        "euler": int(nodes.shape[0] - uniq.shape[0] + tris.shape[0]),
    }
