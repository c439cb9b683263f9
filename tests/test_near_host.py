"""Host logic of the near-field correction against the oracle (CPU only): the
closed-form triangle integral, the index sets and the radius scan of libslp,
called through the C ABI's host-only entry points."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct, nearfield as nfo
from synth import cube, cube_volume_nodes, workloads


def _configurations(rng, count):
    """Triangles with evaluation points in every regime: far, near above the
    face, close to edges and vertices, in the plane inside/outside, on edges
    and at vertices."""
    xs, Ps = [], []
    for k in range(count):
        P = rng.normal(size=(3, 3))
        n = np.cross(P[1] - P[0], P[2] - P[0])
        n /= np.linalg.norm(n)
        bary = rng.dirichlet(np.ones(3))
        inside = bary @ P
        kind = k % 9
        x = {0: inside + 3.0 * rng.normal(size=3),
             1: inside + 1e-3 * n,
             2: 0.5 * (P[0] + P[1]) + 1e-9 * n + 1e-9 * (P[0] - P[2]),
             3: P[1] + 1e-6 * rng.normal(size=3),
             4: inside,
             5: P[0] + 1.7 * (P[1] - P[0]),
             6: 0.3 * P[1] + 0.7 * P[2],
             7: P[2],
             8: inside - 0.4 * (P[0] - inside) + 0.05 * n}[kind]
        xs.append(x)
        Ps.append(P)
    return np.array(xs), np.array(Ps)


def test_triangle_potential_matches_oracle():
    rng = np.random.default_rng(21)
    x, P = _configurations(rng, 900)
    lib = slp.triangle_potential_host(x, P[:, 0], P[:, 1], P[:, 2])
    ref = nfo.triangle_potential(x, P[:, 0], P[:, 1], P[:, 2])
    assert np.all(np.isfinite(lib))
    assert np.allclose(lib, ref, rtol=1e-12, atol=0.0)


def test_triangle_potential_mesh_pairs():
    # every (node, triangle) pair of a small cube mesh, as the near field uses them
    nodes, tris = cube(4)
    x = np.repeat(nodes, tris.shape[0], axis=0)
    T = np.tile(tris, (nodes.shape[0], 1))
    a, b, c = nodes[T[:, 0]], nodes[T[:, 1]], nodes[T[:, 2]]
    lib = slp.triangle_potential_host(x, a, b, c)
    ref = nfo.triangle_potential(x, a, b, c)
    assert np.allclose(lib, ref, rtol=1e-12, atol=0.0)


def _compare_patterns(nodes, tris, targets, eps):
    rp_l, cols_l = slp.near_pattern_host(nodes, tris, targets, eps)
    rp_o, cols_o, dist_o = nfo.near_pairs(nodes, tris, targets, eps)
    A, B, C = (nodes[tris[:, k]] for k in range(3))
    mism = 0
    for i in range(targets.shape[0]):
        a = set(cols_l[rp_l[i]:rp_l[i + 1]].tolist())
        b = set(cols_o[rp_o[i]:rp_o[i + 1]].tolist())
        for j in a ^ b:
            # a pair may only differ on a tie with eps
            d = nfo.point_triangle_distance(targets[i], A[j], B[j], C[j])
            assert abs(d - eps) <= 1e-12 * max(eps, 1.0), (i, j, d, eps)
            mism += 1
        assert np.all(np.diff(cols_l[rp_l[i]:rp_l[i + 1]]) > 0)
    return rp_l[-1], mism


@pytest.mark.parametrize("eps", [0.0, 0.05, 0.3, 0.9, 5.0])
def test_near_pattern_sphere(eps):
    wl = workloads.sphere_uniform(level=2, grid=32, m=4)
    nnz, _ = _compare_patterns(wl.nodes, wl.tris, wl.nodes, eps)
    if eps == 5.0:
        assert nnz == wl.nodes.shape[0] * wl.tris.shape[0]
    if eps == 0.0:
        # only the triangles touching each node
        assert nnz == 3 * wl.tris.shape[0]


@pytest.mark.parametrize("eps", [0.125, 0.2, 0.37])
def test_near_pattern_cube_with_ties(eps):
    # structured mesh: many distances equal eps exactly or within rounding
    nodes, tris = cube(8)
    _compare_patterns(nodes, tris, nodes, eps)


def test_near_pattern_volume_targets():
    nodes, tris = cube(6)
    targets = cube_volume_nodes(6)
    _compare_patterns(nodes, tris, targets, 0.21)


def test_near_radius_matches_oracle():
    wl = workloads.sphere_uniform(level=2, grid=64, m=8)
    prob = direct.prepare_workload(wl)
    for tol in (1e-2, 1e-4, 1e-6):
        ref = nfo.near_radius(prob, tol, wl.es_r_hi)
        got = slp.near_radius_host(prob.omega, prob.gamma, wl.es_r_hi, tol)
        # same scan; the decision at one scan point may flip on rounding
        assert got == pytest.approx(ref, rel=2.1e-3)


def test_near_host_rejects_bad_input():
    nodes, tris = cube(2)
    with pytest.raises(slp.SlpError, match="eps"):
        slp.near_pattern_host(nodes, tris, nodes, -1.0)
    bad = tris.copy()
    bad[0, 0] = nodes.shape[0]
    with pytest.raises(slp.SlpError, match="out of range"):
        slp.near_pattern_host(nodes, bad, nodes, 0.1)
    with pytest.raises(slp.SlpError, match="misses"):
        slp.near_radius_host(np.array([1.0]), np.array([1.0]), 2.0, 1e-6)


def test_near_field_device_bytes_estimate():
    """The host estimate follows the stored layout: rows padded to groups of
    four (short rows), FP64 values, int32 columns, int64 row offsets, one
    element-mean array; every buffer at least 256 bytes."""
    wl = workloads.sphere_uniform(level=2, grid=32, m=4)
    assert slp.near_field_device_bytes(wl.nodes, wl.tris, 0.0) == 0
    a = lambda b: max(b, 256)  # noqa: E731
    for eps in (0.2, 0.6):
        rp, _ = slp.near_pattern_host(wl.nodes, wl.tris, wl.nodes, eps)
        stored = int(((np.diff(rp) + 3) // 4 * 4).sum())
        P, M = wl.nodes.shape[0], wl.tris.shape[0]
        for prec, esz in ((slp.FP64, 8), (slp.FP32, 4)):
            want = a((P + 1) * 8) + a(stored * esz) + a(M * 8) + a(stored * 4)
            assert slp.near_field_device_bytes(wl.nodes, wl.tris, eps, prec) == want
