"""Pins for oracle.direct: R0 (exact kernel), R1 (pair sum), R2 (NDFT). CPU only."""
import copy

import numpy as np
import pytest

from oracle import direct, geometry
from synth import icosphere, density_from_magnetisation, uniform_magnetisation
from synth.workloads import sphere_random, sphere_uniform, make_workload


def _small(level=1, seed=7, grid=(16, 16, 16), m=2):
    wl = sphere_random(level, seed, grid[0], m)
    wl.grid = tuple(grid)
    return direct.prepare_workload(wl)


@pytest.mark.parametrize("grid", [(8, 8, 8), (16, 16, 16), (16, 8, 12), (24, 16, 8)])
def test_pairs_equal_ndft(grid):
    """Exchange of summation order (eq. smooth_phi): R1 == R2 to rounding."""
    p = _small(grid=grid)
    r1 = direct.phi_pairs(p)
    r2 = direct.phi_ndft(p)
    assert np.linalg.norm(r1 - r2) <= 1e-12 * np.linalg.norm(r1)


def test_pairs_equal_ndft_sphere_l3():
    p = direct.prepare_workload(make_workload("sphere_l3"))
    idx = np.arange(0, 642, 9)
    r1 = direct.phi_pairs(p, idx)
    r2 = direct.phi_ndft(p, idx)
    assert np.linalg.norm(r1 - r2) <= 1e-12 * np.linalg.norm(r1)


def test_kernel_against_brute_force_trig_sum():
    """K_F(xi) = Re sum_{l in I_n} c_l e^{2 pi i l.xi} by an explicit loop over the
    asymmetric index set, c_l assembled term by term from the 1-D tables."""
    p = _small(grid=(8, 12, 8))
    rng = np.random.default_rng(3)
    xi = rng.uniform(-0.45, 0.45, size=(6, 3))
    got = direct.fourier_kernel(p, xi)
    n = [int(v) for v in p.n]
    for a in range(xi.shape[0]):
        acc = 0.0 + 0.0j
        for l1 in range(-n[0] // 2, n[0] // 2):
            for l2 in range(-n[1] // 2, n[1] // 2):
                for l3 in range(-n[2] // 2, n[2] // 2):
                    cl = 0.0
                    for t in range(p.omega.size):
                        cl += (p.omega[t] * p.C[0][t, abs(l1)] * p.C[1][t, abs(l2)]
                               * p.C[2][t, abs(l3)])
                    acc += cl * np.exp(2j * np.pi * (l1 * xi[a, 0] + l2 * xi[a, 1] + l3 * xi[a, 2]))
        assert abs(got[a] - acc.real) < 1e-12 * max(1.0, abs(acc.real))


def _with_tables(p, tables, omega):
    q = copy.copy(p)
    q.C = tables
    q.omega = np.asarray(omega, dtype=np.float64)
    return q


def test_dc_only_kernel():
    """c = delta_{l,0}: K_F == 1, so phi = sum_k q_k / (4 pi) at every node."""
    p = _small()
    tabs = [np.zeros((1, int(p.n[q]) // 2 + 1)) for q in range(3)]
    for t in tabs:
        t[0, 0] = 1.0
    q = _with_tables(p, tabs, [1.0])
    ref = p.q.sum() / (4 * np.pi)
    for f in (direct.phi_pairs, direct.phi_ndft):
        assert np.allclose(f(q), ref, rtol=0, atol=1e-15 * np.abs(p.q).sum())


@pytest.mark.parametrize("l0", [(1, 2, 3), (0, 1, 4), (2, 0, 1)])
def test_single_mode_kernel(l0):
    """One cosine pair per axis: tables delta_{|l|,l0_q}. For 0 < l0 < n/2 the axis
    factor is 2 cos(2 pi l0 xi); at l0 = 0 it is 1; at l0 = n/2 it is e^{-i pi n xi}."""
    p = _small(grid=(16, 16, 16))       # n = 8
    n = [int(v) for v in p.n]
    tabs = [np.zeros((1, n[q] // 2 + 1)) for q in range(3)]
    for q in range(3):
        tabs[q][0, l0[q]] = 1.0
    qp = _with_tables(p, tabs, [1.0])
    xt, yt, qq = p.xt, p.yt, p.q
    xi = xt[:, None, :] - yt[None, :, :]
    fac = []
    for q in range(3):
        if l0[q] == 0:
            fac.append(np.ones(xi.shape[:2], dtype=complex))
        elif l0[q] == n[q] // 2:
            fac.append(np.exp(-1j * np.pi * n[q] * xi[..., q]))
        else:
            fac.append(2 * np.cos(2 * np.pi * l0[q] * xi[..., q]) + 0j)
    ref = np.real(fac[0] * fac[1] * fac[2]) @ qq / (4 * np.pi)
    for f in (direct.phi_pairs, direct.phi_ndft):
        assert np.allclose(f(qp), ref, rtol=1e-12, atol=1e-14)


def test_nyquist_mode_closed_form():
    p = _small(grid=(16, 16, 16))
    n = [int(v) for v in p.n]
    tabs = [np.zeros((1, n[q] // 2 + 1)) for q in range(3)]
    tabs[0][0, n[0] // 2] = 1.0
    tabs[1][0, n[1] // 2] = 1.0
    tabs[2][0, 0] = 1.0
    qp = _with_tables(p, tabs, [1.0])
    xi = p.xt[:, None, :] - p.yt[None, :, :]
    # Re(e^{-i pi n xi1} e^{-i pi n xi2}) = cos(pi n (xi1 + xi2))
    ref = np.cos(np.pi * n[0] * (xi[..., 0] + xi[..., 1])) @ p.q / (4 * np.pi)
    for f in (direct.phi_pairs, direct.phi_ndft):
        assert np.allclose(f(qp), ref, rtol=1e-12, atol=1e-14)


def test_linearity_and_reciprocity():
    p = _small()
    rng = np.random.default_rng(5)
    g1, g2 = rng.normal(size=p.g.size), rng.normal(size=p.g.size)
    pa, pb, pc = copy.copy(p), copy.copy(p), copy.copy(p)
    pa.g, pb.g, pc.g = g1, g2, 2.0 * g1 - 3.0 * g2
    ra, rb, rc = (direct.phi_ndft(x) for x in (pa, pb, pc))
    assert np.allclose(rc, 2 * ra - 3 * rb, rtol=1e-12, atol=1e-13 * np.abs(rc).max())
    xi = rng.uniform(-0.4, 0.4, size=(50, 3))
    assert np.allclose(direct.fourier_kernel(p, xi), direct.fourier_kernel(p, -xi), rtol=1e-13)


def test_translation_invariance():
    p = _small()
    q = copy.copy(p)
    shift = np.array([0.013, -0.02, 0.031])        # physical shift of every point
    q.x = p.x + shift
    q.y = p.y + shift
    q.c = p.c + shift
    assert np.allclose(direct.phi_ndft(p), direct.phi_ndft(q), rtol=1e-12, atol=1e-14)


def test_unit_density_sphere():
    """Textbook: a unit single layer on the sphere of radius R has potential R
    inside and on the sphere. R0 converges to it at first order."""
    errs = []
    for L in (2, 3, 4):
        nodes, tris = icosphere(L, 1.0)
        p = direct.prepare(nodes, tris, np.ones(3 * tris.shape[0]), (16, 16, 16), es_r_lo=2e-3,
                           es_r_hi=2.0)
        phi = direct.phi_exact_kernel(p)
        errs.append(np.abs(phi - 1.0).max())
    assert errs[-1] < 2.5e-2
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6


def test_uniformly_magnetised_sphere():
    """Interior potential x3/3 for m = (0,0,1), R = 1 (eq. phi_anal); the paper
    observes linear decay of the nodal error with the mesh size."""
    errs = []
    for L in (2, 3, 4):
        nodes, tris = icosphere(L, 1.0)
        g = density_from_magnetisation(nodes, tris, uniform_magnetisation())
        p = direct.prepare(nodes, tris, g, (16, 16, 16), es_r_lo=2e-3, es_r_hi=2.0)
        errs.append(np.abs(direct.phi_exact_kernel(p) - nodes[:, 2] / 3).max())
    assert errs[-1] < 5e-3
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6


def test_radial_magnetisation_gives_zero_density():
    """m = x/|x| on a sphere with dphi1/dn = 1 gives g = 0 and phi_2 = 0 (Sec. 4)."""
    nodes, tris = icosphere(2)
    y, _ = geometry.quadrature(nodes, tris)
    _, nrm = geometry.triangle_areas_normals(nodes, tris)
    mdotn = np.einsum("kd,kd->k", y / np.linalg.norm(y, axis=1, keepdims=True), np.tile(nrm, (3, 1)))
    # flat triangles: m.n is not exactly 1, g = m.n - dphi1/dn vanishes up to O(h^2)
    g = mdotn - np.tile(np.einsum("kd,kd->k",
                                  (y / np.linalg.norm(y, axis=1, keepdims=True))[:tris.shape[0]],
                                  nrm), 3)
    p = direct.prepare(nodes, tris, np.zeros_like(g), (16, 16, 16), es_r_lo=2e-3, es_r_hi=2.0)
    assert np.all(direct.phi_ndft(p) == 0.0)


def test_targets_off_the_surface_both_routes():
    """R1 (pair sum) and R2 (NDFT) agree at volume lattice points inside the
    cube, and at the nodes the targets option gives the default result."""
    from synth import cube, cube_volume_nodes, RandomSmoothMagnetisation, density_from_magnetisation
    nodes, tris = cube(4)
    mf = RandomSmoothMagnetisation(17, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    from synth.workloads import expsum_interval
    r_lo, r_hi = expsum_interval(nodes)
    kw = dict(es_r_lo=r_lo, es_r_hi=r_hi)
    tg = cube_volume_nodes(4)
    p = direct.prepare(nodes, tris, dens, (32, 32, 32), targets=tg, **kw)
    a, b = direct.phi_pairs(p), direct.phi_ndft(p)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    p0 = direct.prepare(nodes, tris, dens, (32, 32, 32), **kw)
    p1 = direct.prepare(nodes, tris, dens, (32, 32, 32), targets=nodes, **kw)
    assert np.array_equal(direct.phi_ndft(p0), direct.phi_ndft(p1))
