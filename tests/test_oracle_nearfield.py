"""Pins for oracle.nearfield (CPU only): the exact triangle integrals against
closed forms, brute-force quadrature and the paper's singular-case rule; the
distance and index sets against brute force; the near-field correction against
the exact surface integrals and the uniformly magnetised sphere."""
import numpy as np
import pytest
from scipy import integrate

from oracle import direct, nearfield as nfo
from synth import workloads

LN = np.log(1.0 + np.sqrt(2.0))


def _brute_potential(x, P):
    """Adaptive 2-D quadrature of 1/|x - y| over the triangle's parameter domain."""
    e1, e2 = P[1] - P[0], P[2] - P[0]
    J = np.linalg.norm(np.cross(e1, e2))
    f = lambda v, u: J / np.linalg.norm(x - (P[0] + u * e1 + v * e2))  # noqa: E731
    return integrate.dblquad(f, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=1e-14, epsrel=1e-13)[0]


def _children(P):
    a, b, c = P
    ab, bc, ca = 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)
    return [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]


def test_square_centre_closed_form():
    # unit density on a square of side a, at its centre: 4 a ln(1 + sqrt 2)
    for a in (1.0, 0.37):
        O, A, B, C = (np.array(v, dtype=float) * a for v in ([0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]))
        ctr = 0.5 * (O + B)
        I = nfo.triangle_potential(ctr, O, A, B) + nfo.triangle_potential(ctr, O, B, C)
        assert I == pytest.approx(4.0 * a * LN, rel=1e-14)


def test_right_isosceles_vertices_closed_form():
    # legs a: at the right-angle vertex sqrt(2) a ln(1 + sqrt 2), at a 45-degree vertex a ln(1 + sqrt 2)
    a = 0.8
    O, A, B = np.zeros(3), np.array([a, 0.0, 0.0]), np.array([0.0, a, 0.0])
    assert nfo.triangle_potential(O, O, A, B) == pytest.approx(np.sqrt(2.0) * a * LN, rel=1e-14)
    assert nfo.triangle_potential(A, O, A, B) == pytest.approx(a * LN, rel=1e-14)
    assert nfo.triangle_potential(B, O, A, B) == pytest.approx(a * LN, rel=1e-14)


def test_vertex_case_matches_paper_duffy_rule():
    rng = np.random.default_rng(11)
    for _ in range(10):
        P = rng.normal(size=(3, 3))
        for v in range(3):
            apex, p1, p2 = P[v], P[(v + 1) % 3], P[(v + 2) % 3]
            ref = nfo.vertex_potential_duffy(apex, p1, p2, order=96)
            assert nfo.triangle_potential(apex, *P) == pytest.approx(ref, rel=1e-10)


def test_against_brute_force_quadrature():
    rng = np.random.default_rng(12)
    for _ in range(8):
        P = rng.normal(size=(3, 3))
        x = P.mean(axis=0) + rng.normal(size=3)
        assert nfo.triangle_potential(x, *P) == pytest.approx(_brute_potential(x, P), rel=1e-11)


@pytest.mark.parametrize("where", ["above_centroid", "near_edge_midpoint", "on_edge_line_outside",
                                   "in_plane_outside", "in_plane_inside", "on_edge", "at_vertex"])
def test_additive_under_midpoint_subdivision(where):
    rng = np.random.default_rng(13)
    for _ in range(5):
        P = rng.normal(size=(3, 3))
        n = np.cross(P[1] - P[0], P[2] - P[0])
        n /= np.linalg.norm(n)
        x = {"above_centroid": P.mean(0) + 1e-3 * n,
             "near_edge_midpoint": 0.5 * (P[0] + P[1]) + 1e-7 * n,
             "on_edge_line_outside": P[0] + 2.0 * (P[1] - P[0]),
             "in_plane_outside": 0.3 * P[0] + 0.7 * P[1] + 0.2 * (P[1] - P[2]),
             "in_plane_inside": 0.2 * P[0] + 0.3 * P[1] + 0.5 * P[2],
             "on_edge": 0.25 * P[1] + 0.75 * P[2],
             "at_vertex": P[2]}[where]
        whole = nfo.triangle_potential(x, *P)
        parts = sum(nfo.triangle_potential(x, *k) for k in _children(P))
        assert parts == pytest.approx(whole, rel=1e-12)


def test_invariant_under_vertex_order_and_rigid_motion():
    rng = np.random.default_rng(14)
    P = rng.normal(size=(3, 3))
    x = P.mean(0) + 0.1 * rng.normal(size=3)
    ref = nfo.triangle_potential(x, *P)
    for perm in ([0, 2, 1], [1, 0, 2], [2, 1, 0], [1, 2, 0]):
        assert nfo.triangle_potential(x, *P[perm]) == pytest.approx(ref, rel=1e-13)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    sh = rng.normal(size=3)
    assert nfo.triangle_potential(Q @ x + sh, *(P @ Q.T + sh)) == pytest.approx(ref, rel=1e-12)


def test_far_field_is_area_over_distance():
    rng = np.random.default_rng(15)
    P = rng.normal(size=(3, 3))
    c = P.mean(0)
    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    L = np.linalg.norm(P - c, axis=1).max()
    for r in (10.0, 100.0, 1000.0):
        u = rng.normal(size=3)
        x = c + r * u / np.linalg.norm(u)
        # the dipole term vanishes about the centroid: relative error <= (L / r)^2
        assert abs(nfo.triangle_potential(x, *P) * r / area - 1.0) <= (L / r) ** 2


def test_distance_against_sampling():
    rng = np.random.default_rng(16)
    g = np.linspace(0.0, 1.0, 401)
    U, V = np.meshgrid(g, g)
    keep = U + V <= 1.0
    U, V = U[keep], V[keep]
    for _ in range(30):
        P = rng.normal(size=(3, 3))
        x = P.mean(0) + 1.5 * rng.normal(size=3)
        pts = P[0] + U[:, None] * (P[1] - P[0]) + V[:, None] * (P[2] - P[0])
        brute = np.linalg.norm(pts - x, axis=1).min()
        d = nfo.point_triangle_distance(x, *P)
        h = 2.0 * np.linalg.norm(P - P.mean(0), axis=1).max() / 400.0
        assert d <= brute + 1e-14 and brute - d <= h


def test_distance_special_cases():
    a, b, c = np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    assert nfo.point_triangle_distance(np.array([0.2, 0.2, -0.7]), a, b, c) == pytest.approx(0.7)
    assert nfo.point_triangle_distance(np.array([-3.0, -4.0, 0.0]), a, b, c) == pytest.approx(5.0)
    assert nfo.point_triangle_distance(np.array([0.5, -2.0, 0.0]), a, b, c) == pytest.approx(2.0)
    assert nfo.point_triangle_distance(np.array([1.0, 1.0, 0.0]), a, b, c) == pytest.approx(np.sqrt(0.5))
    assert nfo.point_triangle_distance(c, a, b, c) == 0.0


def test_near_pairs_match_distances():
    wl = workloads.sphere_uniform(level=1, grid=32, m=4)
    eps = 0.6
    rowptr, cols, dist = nfo.near_pairs(wl.nodes, wl.tris, wl.nodes, eps)
    A, B, C = (wl.nodes[wl.tris[:, k]] for k in range(3))
    for i in range(wl.nodes.shape[0]):
        d = nfo.point_triangle_distance(wl.nodes[i][None], A, B, C)
        row = cols[rowptr[i]:rowptr[i + 1]]
        assert np.array_equal(row, np.nonzero(d <= eps)[0])
        # every triangle touching node i is at distance 0
        touching = np.nonzero((wl.tris == i).any(axis=1))[0]
        assert np.all(np.isin(touching, row))
    assert np.all(dist <= eps)


def test_near_radius_brackets_tolerance():
    wl = workloads.sphere_uniform(level=2, grid=64, m=8)
    prob = direct.prepare_workload(wl)
    for tol in (1e-2, 1e-4, 1e-6):
        eps = nfo.near_radius(prob, tol, wl.es_r_hi)
        err = lambda r: abs(nfo.smooth_kernel(prob, np.array([r]))[0] * r - 1.0)  # noqa: E731
        assert err(eps) <= tol < err(eps * 0.999)
        # 1/r is matched on the whole scan above eps
        rs = np.geomspace(eps, wl.es_r_hi, 300)
        assert max(err(r) for r in rs) <= tol * 1.0001


@pytest.fixture(scope="module")
def sphere2():
    wl = workloads.sphere_uniform(level=2, grid=64, m=8)
    prob = direct.prepare_workload(wl)
    gbar = nfo.element_mean_density(prob, wl.tris.shape[0])
    exact = nfo.phi_exact_integrals(wl.nodes, wl.tris, gbar, wl.nodes)
    far = direct.phi_pairs(prob)
    return wl, prob, exact, far


def test_exact_integrals_uniformly_magnetised_sphere():
    # phi_2 = z / 3 on the sphere for m = e_z (closed form of the Numerics section);
    # the flat-triangle error is O(h^2): halving h divides it by about 4
    errs = []
    for level in (1, 2):
        wl = workloads.sphere_uniform(level=level, grid=64, m=8)
        prob = direct.prepare_workload(wl)
        gbar = nfo.element_mean_density(prob, wl.tris.shape[0])
        ex = nfo.phi_exact_integrals(wl.nodes, wl.tris, gbar, wl.nodes)
        errs.append(np.abs(ex - wl.nodes[:, 2] / 3.0).max())
    assert errs[1] < 7e-3 and 3.0 < errs[0] / errs[1] < 5.5


def test_near_field_completes_the_smooth_part(sphere2):
    wl, prob, exact, far = sphere2
    scale = np.abs(exact).max()
    # the smooth part alone is far off on this grid
    assert np.abs(far - exact).max() > 0.1 * scale
    eps = nfo.near_radius(prob, 1e-3, wl.es_r_hi)
    near, rowptr, cols, vals = nfo.phi_near(prob, wl.nodes, wl.tris, eps)
    assert 0 < cols.size < wl.nodes.shape[0] * wl.tris.shape[0]
    # left over: the Fourier error of the smooth kernel and the three-point
    # rule on the far pairs
    assert np.abs(far + near - exact).max() < 1e-4 * scale


def test_near_field_over_all_pairs_leaves_only_fourier_error(sphere2):
    wl, prob, exact, far = sphere2
    near, *_ = nfo.phi_near(prob, wl.nodes, wl.tris, 1e9)
    # every pair corrected: phi_s + phi_NF - exact = 1/(4 pi) sum w g (K_F - N_s)
    M = wl.tris.shape[0]
    xi = (wl.nodes[:, None, :] - prob.y[None, :, :]).reshape(-1, 3)
    kf = direct.fourier_kernel(prob, xi * prob.s[None, :])
    ns = nfo.smooth_kernel(prob, np.linalg.norm(xi, axis=1))
    resid = ((kf - ns).reshape(wl.nodes.shape[0], 3 * M) @ prob.q) / nfo.FOUR_PI
    assert np.allclose(far + near - exact, resid, rtol=0.0, atol=1e-12 * np.abs(exact).max())
