"""Pins for oracle.geometry and the synthetic meshes (CPU only)."""
import numpy as np
import pytest

from oracle import geometry
from synth import icosphere, cube, thin_film, mesh_summary, box_surface


def _tri_second_moments(P):
    """Closed form int_T x_i x_j dA = A/12 (sum_a P_ai P_aj + (sum_a P_ai)(sum_b P_bj))
    from int lambda_a lambda_b dA = A (1 + delta_ab) / 12."""
    A = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    S = P.sum(axis=0)
    return A, A / 12.0 * (P.T @ P + np.outer(S, S))


def test_quadrature_exact_for_quadratics():
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = rng.normal(size=(3, 3))
        y, w = geometry.quadrature(P, np.array([[0, 1, 2]], dtype=np.int32))
        A, mom2 = _tri_second_moments(P)
        assert np.isclose(w.sum(), A, rtol=1e-14)
        # first moments: A * centroid
        assert np.allclose(w @ y, A * P.mean(axis=0), rtol=1e-13, atol=1e-14)
        # second moments: exact for the degree-2 rule
        assert np.allclose((w[:, None] * y).T @ y, mom2, rtol=1e-12, atol=1e-14)


def test_long_index_order():
    nodes, tris = icosphere(1)
    y, w = geometry.quadrature(nodes, tris)
    M = tris.shape[0]
    cen = nodes[tris].mean(axis=1)
    for s in range(3):
        # point s lies halfway between the centroid and vertex s of triangle j
        assert np.allclose(y[s * M:(s + 1) * M] - cen, 0.5 * (nodes[tris[:, s]] - cen))


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts(level):
    nodes, tris = icosphere(level)
    s = mesh_summary(nodes, tris)
    assert s["tris"] == 20 * 4 ** level and s["nodes"] == 10 * 4 ** level + 2
    assert s["every_edge_shared_twice"] and s["euler"] == 2
    assert np.allclose(np.linalg.norm(nodes, axis=1), 1.0)


def test_box_counts_and_closedness():
    nodes, tris = cube(64)
    s = mesh_summary(nodes, tris)
    assert (s["nodes"], s["tris"]) == (24578, 49152)
    assert s["every_edge_shared_twice"] and s["euler"] == 2
    area, nrm = geometry.triangle_areas_normals(nodes, tris)
    assert np.isclose(area.sum(), 6.0, rtol=1e-13)
    # closed surface: the integral of the normal vanishes
    assert np.allclose((area[:, None] * nrm).sum(0), 0.0, atol=1e-12)
    # outward: normal . (centroid - centre) > 0
    cen = nodes[tris].mean(axis=1)
    assert np.all(np.einsum("ij,ij->i", nrm, cen) > 0)


def test_film_counts():
    nodes, tris = thin_film(512, 10)
    assert nodes.shape[0] == 544770 and tris.shape[0] == 1089536
    area, _ = geometry.triangle_areas_normals(nodes, tris)
    assert np.isclose(area.sum(), 2 * 1.0 + 4 * 0.02, rtol=1e-12)


def test_sphere_area_converges():
    errs = []
    for L in range(1, 5):
        nodes, tris = icosphere(L)
        area, _ = geometry.triangle_areas_normals(nodes, tris)
        errs.append(abs(area.sum() - 4 * np.pi))
    # inscribed polyhedron: second order in the mesh size
    assert all(errs[i + 1] < errs[i] / 3.5 for i in range(len(errs) - 1))


@pytest.mark.parametrize("grid", [(64, 64, 64), (128, 128, 128), (1024, 1024, 64), (32, 16, 8)])
def test_scaling_rule(grid):
    nodes, _ = box_surface((1.0, 0.5, 0.02), (8, 4, 2))
    c, s = geometry.scaling(nodes, grid)
    xt = geometry.to_torus(nodes, c, s)
    assert np.all(np.abs(xt) <= 0.2 + 1e-15)
    # equal physical grid spacing on every axis: s_q N_q constant
    sN = s * np.asarray(grid)
    assert np.allclose(sN, sN[0], rtol=1e-15)
    # the limiting axis touches the box boundary
    assert np.isclose(np.abs(xt).max(), 0.2, rtol=1e-14)


def _closed_volume(nodes, tris):
    """Volume of a closed, outward-oriented polyhedron: (1/6) sum p0 . (p1 x p2)."""
    p = nodes[tris]
    return np.einsum("ij,ij->i", p[:, 0], np.cross(p[:, 1], p[:, 2])).sum() / 6.0


def test_density_p1_constant_and_affine_fields():
    nodes, tris = icosphere(2)
    M = tris.shape[0]
    _, nrm = geometry.triangle_areas_normals(nodes, tris)
    # constant m: g_j = m . n_j
    mc = np.array([0.3, -0.2, 0.9])
    g = geometry.density_p1(nodes, tris, np.tile(mc, (nodes.shape[0], 1)))
    assert np.allclose(g[:M], nrm @ mc, rtol=0, atol=1e-15)
    assert np.array_equal(g[:M], g[M:2 * M]) and np.array_equal(g[:M], g[2 * M:])
    # affine m(x) = A x + b: the integral mean is the value at the centroid
    rng = np.random.default_rng(3)
    A, b = rng.normal(size=(3, 3)), rng.normal(size=3)
    g = geometry.density_p1(nodes, tris, nodes @ A.T + b)
    cen = nodes[tris].mean(axis=1)
    assert np.allclose(g[:M], ((cen @ A.T + b) * nrm).sum(axis=1), rtol=0, atol=1e-13)
    # dphi1/dn is subtracted per triangle
    d = rng.normal(size=M)
    g2 = geometry.density_p1(nodes, tris, nodes @ A.T + b, d)
    assert np.allclose(g2[:M], g[:M] - d, rtol=0, atol=1e-15)


@pytest.mark.parametrize("mesh", ["sphere", "cube"])
def test_density_p1_divergence_theorem(mesh):
    """sum_j |S_j| g_j = int_{dOmega} m.n = int_Omega div m: 0 for a uniform m,
    3 Vol for m(x) = x (exact on the polyhedron: m is affine, the faces flat)."""
    nodes, tris = icosphere(3) if mesh == "sphere" else cube(6)
    area, _ = geometry.triangle_areas_normals(nodes, tris)
    M = tris.shape[0]
    g = geometry.density_p1(nodes, tris, np.tile([0.0, 0.0, 1.0], (nodes.shape[0], 1)))
    assert abs(area @ g[:M]) < 1e-13
    vol = _closed_volume(nodes, tris)
    g = geometry.density_p1(nodes, tris, nodes)
    assert np.isclose(area @ g[:M], 3.0 * vol, rtol=1e-13)


def test_cube_volume_nodes():
    from synth import cube_volume_nodes
    for c in (2, 5, 16):
        v = cube_volume_nodes(c)
        assert v.shape == ((c + 1) ** 3, 3)
        nodes, _ = cube(c)
        on_boundary = v[np.any(np.isclose(np.abs(v), 0.5), axis=1)]
        key = lambda a: set(map(tuple, np.round(a * 2 * c).astype(int)))
        assert key(on_boundary) == key(nodes)
