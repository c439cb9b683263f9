"""Pins for oracle.fem (CPU only): the P1 stiffness matrix and load vector, the
Dirichlet solve against exact and manufactured solutions, the normal
derivative, the boundary faces, and the complete scalar potential of Alg. 1
against the closed forms of the Numerics section."""
import numpy as np
import pytest

from oracle import direct, fem, nearfield as nfo
from synth import ball_tets, cube, cube_tets
from synth.workloads import expsum_interval


def _manufactured(nodes):
    """phi_e = (1/4 - x^2)(1/4 - y^2)(1/4 - z^2) vanishes on the unit cube's
    boundary; with m = grad phi_e the exact scalar potential is phi_e inside (it
    solves -Laplace phi = -div m with the jump [d phi/dn] = -m.n and phi = 0
    outside)."""
    x, y, z = nodes.T
    ax, ay, az = 0.25 - x * x, 0.25 - y * y, 0.25 - z * z
    m = np.stack([-2 * x * ay * az, -2 * y * ax * az, -2 * z * ax * ay], axis=1)
    return ax * ay * az, m


def test_reference_element():
    n = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    t = np.array([[0, 1, 2, 3]], dtype=np.int32)
    want = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1.0]]) / 6.0
    assert np.allclose(fem.stiffness(n, t).toarray(), want, atol=1e-15)
    vol, G = fem.tet_gradients(n, t)
    assert vol[0] == pytest.approx(1.0 / 6.0)


def test_stiffness_properties():
    nodes, tets = cube_tets(5)
    S = fem.stiffness(nodes, tets)
    vol, _ = fem.tet_gradients(nodes, tets)
    assert vol.sum() == pytest.approx(1.0, rel=1e-13) and np.all(vol > 0)
    assert abs(S - S.T).max() < 1e-14
    assert np.abs(S @ np.ones(nodes.shape[0])).max() < 1e-13
    v = np.random.default_rng(1).normal(size=nodes.shape[0])
    assert v @ (S @ v) > 0
    # the energy of a linear function a.x is |a|^2 times the volume
    a = np.array([0.3, -1.2, 0.7])
    u = nodes @ a
    assert u @ (S @ u) == pytest.approx(a @ a, rel=1e-12)


def test_linear_dirichlet_data_reproduced_exactly():
    nodes, tets = cube_tets(6)
    S = fem.stiffness(nodes, tets)
    bnd = fem.boundary_nodes(tets, nodes)
    u = nodes @ np.array([0.4, -0.9, 1.3]) + 0.25
    x = fem.solve_dirichlet(S, np.zeros(nodes.shape[0]), bnd, u[bnd])
    assert np.abs(x - u).max() < 1e-12


def test_iterative_solve_matches_direct():
    nodes, tets = ball_tets(8)
    r = np.linalg.norm(nodes, axis=1)
    m = nodes / np.where(r > 0, r, 1.0)[:, None]
    a = fem.solve_phi1(nodes, tets, m, "direct")
    b = fem.solve_phi1(nodes, tets, m, "cg")
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()


def test_uniform_magnetisation_gives_zero_phi1():
    nodes, tets = ball_tets(6)
    m = np.tile([0.2, -0.5, 1.0], (nodes.shape[0], 1))
    b = fem.load(nodes, tets, m)
    free = ~fem.boundary_nodes(tets, nodes)
    assert np.abs(b[free]).max() < 1e-15
    assert np.abs(fem.solve_phi1(nodes, tets, m)).max() < 1e-14


def test_manufactured_solution_converges():
    errs, derrs = [], []
    for c in (8, 16):
        nodes, tets = cube_tets(c)
        phie, m = _manufactured(nodes)
        phi1 = fem.solve_phi1(nodes, tets, m)
        tris, own = fem.boundary_faces(nodes, tets)
        dn = fem.dphi1_dn(nodes, tets, phi1, tris, own)
        cen = nodes[tris].mean(axis=1)
        _, mc = _manufactured(cen)
        nrm = np.cross(nodes[tris[:, 1]] - nodes[tris[:, 0]], nodes[tris[:, 2]] - nodes[tris[:, 0]])
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        errs.append(np.abs(phi1 - phie).max())
        derrs.append(np.abs(dn - np.einsum("ij,ij->i", mc, nrm)).max())
    assert errs[1] < 2e-4 and errs[0] / errs[1] > 3.5          # O(h^2) at the nodes
    assert derrs[1] < 1.1e-2 and derrs[0] / derrs[1] > 1.7     # O(h) gradient


def test_boundary_faces_are_the_cube_surface():
    for c in (3, 8):
        nodes, tets = cube_tets(c)
        tris, own = fem.boundary_faces(nodes, tets)
        sn, st = cube(c)
        key = lambda P: {tuple(sorted(map(tuple, np.round(f * 1e6).astype(int)))) for f in P}  # noqa: E731
        assert key(nodes[tris]) == key(sn[st]) and tris.shape[0] == st.shape[0]
        # outward: normal . (centroid - centre) > 0 on the convex cube
        n = np.cross(nodes[tris[:, 1]] - nodes[tris[:, 0]], nodes[tris[:, 2]] - nodes[tris[:, 0]])
        assert np.all(np.einsum("ij,ij->i", n, nodes[tris].mean(axis=1)) > 0)
        # each face is a face of its owner
        assert all(set(f) <= set(tets[o]) for f, o in zip(tris.tolist(), own.tolist()))


def test_ball_mesh_and_radial_magnetisation():
    # m = x/|x| in the ball of radius R: phi = |x| - R inside (Numerics section);
    # phi_2 = 0, so phi_1 alone converges to it (first order on these meshes)
    errs = []
    for c in (8, 16):
        nodes, tets = ball_tets(c, 1.0)
        vol, _ = fem.tet_gradients(nodes, tets)
        assert np.all(vol > 0)
        tris, _ = fem.boundary_faces(nodes, tets)
        assert np.allclose(np.linalg.norm(nodes[np.unique(tris)], axis=1), 1.0)
        r = np.linalg.norm(nodes, axis=1)
        m = nodes / np.where(r > 0, r, 1.0)[:, None]
        errs.append(np.abs(fem.solve_phi1(nodes, tets, m) - (r - 1.0)).max())
    assert errs[1] < 0.1 and errs[0] / errs[1] > 1.7


def _eps(nodes, tets, grid, tol):
    lo, hi = expsum_interval(nodes)
    tris, _ = fem.boundary_faces(nodes, tets)
    prob = direct.prepare(nodes, tris, np.zeros(3 * tris.shape[0]), grid, es_r_lo=lo, es_r_hi=hi)
    return nfo.near_radius(prob, tol, hi), lo, hi


def test_scalar_potential_uniformly_magnetised_ball():
    # m = e_z: phi_1 = 0 and phi = phi_2 = z/3 at every node, interior ones too;
    # phi_2 also matches the exact surface integrals of its density
    nodes, tets = ball_tets(8, 1.0)
    m = np.tile([0.0, 0.0, 1.0], (nodes.shape[0], 1))
    grid = (64, 64, 64)
    eps, lo, hi = _eps(nodes, tets, grid, 1e-3)
    phi, phi1, phi2, dn, tris = fem.scalar_potential(nodes, tets, m, grid, eps, es_r_lo=lo,
                                                     es_r_hi=hi, parts=True)
    assert np.abs(phi1).max() < 1e-14 and np.abs(dn).max() < 1e-12
    assert np.abs(phi - nodes[:, 2] / 3.0).max() < 5e-3
    gbar = np.einsum("tki,ti->t", m[tris], np.cross(nodes[tris[:, 1]] - nodes[tris[:, 0]],
                                                   nodes[tris[:, 2]] - nodes[tris[:, 0]])) / 3.0
    gbar /= np.linalg.norm(np.cross(nodes[tris[:, 1]] - nodes[tris[:, 0]],
                                    nodes[tris[:, 2]] - nodes[tris[:, 0]]), axis=1)
    exact = nfo.phi_exact_integrals(nodes, tris, gbar, nodes)
    # left over: the Fourier error N_s - K_F of the smooth part (~1e-4 on this grid)
    assert np.abs(phi2 - exact).max() < 3e-4 * np.abs(exact).max()


def test_scalar_potential_manufactured_cube():
    # m = grad phi_e: phi = phi_e; phi_1 carries it, phi_2 (density m.n - dphi_1/dn,
    # a discretisation residual) is small
    nodes, tets = cube_tets(8)
    phie, m = _manufactured(nodes)
    grid = (64, 64, 64)
    eps, lo, hi = _eps(nodes, tets, grid, 1e-3)
    phi, phi1, phi2, dn, tris = fem.scalar_potential(nodes, tets, m, grid, eps, es_r_lo=lo,
                                                     es_r_hi=hi, parts=True)
    assert np.abs(phi1 - phie).max() < 1e-3
    assert np.abs(phi - phie).max() < 6e-3 and np.abs(phi2).max() < 6e-3


def test_prism_demag_factor_closed_form():
    # the cube: 1/3 by symmetry; any prism: the three factors sum to 1; a thin
    # plate tends to 1 across its thickness
    assert fem.prism_demag_factor(1.0, 1.0, 1.0) == pytest.approx(1.0 / 3.0, abs=1e-14)
    rng = np.random.default_rng(31)
    for _ in range(5):
        a, b, c = rng.uniform(0.1, 3.0, size=3)
        s = fem.prism_demag_factor(a, b, c) + fem.prism_demag_factor(b, c, a) + fem.prism_demag_factor(c, a, b)
        assert s == pytest.approx(1.0, abs=1e-12)
    thin = [fem.prism_demag_factor(1.0, 1.0, c) for c in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)]
    assert np.all(np.diff(thin) > 0) and thin[-1] > 0.9999
    # the reference energy printed with Table 3 (film 1 x 1 x 0.1 magnetised across)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table3_film_energy.txt")
    ref = float([l for l in open(path) if not l.startswith("#")][0])
    assert 0.5 * fem.prism_demag_factor(0.5, 0.5, 0.05) * 0.1 == pytest.approx(ref, abs=5e-6)


def test_energy_uniform_film_and_ball():
    # Alg. 1 followed by E = (1/2) int m . grad phi against the closed forms:
    # the 1 x 1 x 0.1 film magnetised across (N V / 2) and the ball (V / 6)
    from synth import box_tets
    grid = (64, 64, 32)
    nodes, tets = box_tets((1.0, 1.0, 0.1), (16, 16, 2))
    m = np.tile([0.0, 0.0, 1.0], (nodes.shape[0], 1))
    eps, lo, hi = _eps(nodes, tets, grid, 1e-3)
    phi = fem.scalar_potential(nodes, tets, m, grid, eps, es_r_lo=lo, es_r_hi=hi)
    E = fem.stray_field_energy(nodes, tets, m, phi)
    assert abs(E / (0.5 * fem.prism_demag_factor(0.5, 0.5, 0.05) * 0.1) - 1.0) < 0.02
    errs = []
    for c in (6, 8):
        nodes, tets = ball_tets(c, 1.0)
        m = np.tile([0.0, 0.0, 1.0], (nodes.shape[0], 1))
        eps, lo, hi = _eps(nodes, tets, (64, 64, 64), 1e-3)
        phi = fem.scalar_potential(nodes, tets, m, (64, 64, 64), eps, es_r_lo=lo, es_r_hi=hi)
        vol, _ = fem.tet_gradients(nodes, tets)
        errs.append(abs(fem.stray_field_energy(nodes, tets, m, phi) / (vol.sum() / 6.0) - 1.0))
    assert errs[1] < 0.015 and errs[1] < errs[0]
