"""Pins of the oracle's integrated-window gridding (Sec. 3.1, eq. gridding2):
the collapsed Gauss rule against the exact moments of the unit triangle, the
closed-form Fourier transform of a triangle against scipy's adaptive double
integral, the gridding after deconvolution (eq. deconv) against the closed
form on every well-conditioned mode, and additivity under subdivision."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import direct, integrated as iw, nufft
from synth import workloads


def test_duffy_rule_moments():
    # int over the unit triangle of xi1^a xi2^b = a! b! / (a + b + 2)!
    for n in (3, 6, 12):
        xi, w = iw.duffy_rule(n)
        assert w.sum() == pytest.approx(0.5, abs=1e-15)
        for a in range(0, 2 * n - 1):
            for b in range(0, 2 * n - 1 - a):
                exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
                got = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b)
                assert got == pytest.approx(exact, rel=1e-12, abs=1e-16), (n, a, b)


def _problem(level=2, grid=32, m=6):
    wl = workloads.sphere_uniform(level=level, grid=grid, m=m)
    return wl, direct.prepare_workload(wl)


def test_exp_divided_difference_branches():
    """Series and difference-quotient branches of the stable second divided
    difference agree where both apply, and l = 0 gives the area."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, size=(3, 200))
    dd = iw._exp_dd2(*x)
    f = lambda v: np.exp(-1j * v)  # noqa: E731
    ref = ((f(x[2]) - f(x[1])) / (x[2] - x[1]) - (f(x[1]) - f(x[0])) / (x[1] - x[0])) / (x[2] - x[0])
    ok = np.min(np.abs(np.stack([x[0] - x[1], x[1] - x[2], x[0] - x[2]])), axis=0) > 0.3
    assert np.allclose(dd[ok], ref[ok], rtol=1e-12, atol=1e-13)
    c = rng.uniform(-3, 3, size=50)
    near = iw._exp_dd2(c, c + 1e-4, c + 2e-4)
    assert np.allclose(near, -0.5 * f(c + 1e-4), rtol=1e-7)   # f''/2 at the cluster
    wl, prob = _problem()
    F = iw.triangle_fourier(prob, wl.nodes, wl.tris, (0, 0, 0))
    P0, P1, P2 = (wl.nodes[wl.tris[:, k]] for k in range(3))
    assert np.allclose(F, 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0), axis=1), rtol=1e-14)


def test_triangle_fourier_against_adaptive_quadrature():
    wl, prob = _problem()
    tris = wl.tris[:5]
    rng = np.random.default_rng(3)
    for _ in range(4):
        l = rng.integers(-8, 8, size=3)
        F = iw.triangle_fourier(prob, wl.nodes, tris, l)
        for j in range(tris.shape[0]):
            P = [np.asarray(wl.nodes[tris[j, k]]) for k in range(3)]
            area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))

            def f(x2, x1, part):
                y = P[0] + x1 * (P[1] - P[0]) + x2 * (P[2] - P[0])
                ph = -2 * np.pi * np.dot((y - prob.c) * prob.s, l)
                return (np.cos(ph) if part == 0 else np.sin(ph)) * 2 * area

            re = integrate.dblquad(f, 0, 1, 0, lambda x1: 1 - x1, args=(0,), epsabs=1e-14, epsrel=1e-12)[0]
            im = integrate.dblquad(f, 0, 1, 0, lambda x1: 1 - x1, args=(1,), epsabs=1e-14, epsrel=1e-12)[0]
            assert abs(F[j] - (re + 1j * im)) <= 1e-9 * area, (l, j)


@pytest.mark.parametrize("window,m,tol", [("kb", 6, 1e-9), ("gauss", 8, 1e-6)])
def test_gridding_deconvolves_to_triangle_transform(window, m, tol):
    """c_l(f) / c_l(Upsilon~) of the integrated gridding equals
    sum_j g_j int_{S_j} exp(-2 pi i y~.l) dsigma up to the window error
    (eq. deconv), on every mode whose closed form is well conditioned."""
    wl, prob = _problem(m=m)
    M = wl.tris.shape[0]
    a = iw.gridding_integrated(prob, wl.nodes, wl.tris, m, window, n=12)
    b = nufft.spectrum_b(prob, a, m, window)
    gj = iw.element_density(prob, M)
    n = [int(v) for v in prob.n]
    ls = [np.arange(-k // 2, k // 2) for k in n]
    errs, scale = [], np.abs(b).max()
    for i0, l0 in enumerate(ls[0]):
        for i1, l1 in enumerate(ls[1]):
            for i2, l2 in enumerate(ls[2]):
                F = iw.triangle_fourier(prob, wl.nodes, wl.tris, (l0, l1, l2))
                errs.append(abs(b[i0, i1, i2] - np.dot(gj, F)))
    assert max(errs) <= tol * scale


def test_gridding_is_additive_under_subdivision():
    """Splitting every triangle into its four midpoint children (same element
    density) leaves the integrated gridding unchanged."""
    wl, prob = _problem(m=6)
    nodes, tris = wl.nodes, wl.tris
    M = tris.shape[0]
    a = iw.gridding_integrated(prob, nodes, tris, 6, "kb", n=12)
    mids, kids, gk = [], [], []
    base = nodes.shape[0]
    gj = iw.element_density(prob, M)
    for j, (i0, i1, i2) in enumerate(tris):
        m01, m12, m20 = base + 3 * j, base + 3 * j + 1, base + 3 * j + 2
        mids += [(nodes[i0] + nodes[i1]) / 2, (nodes[i1] + nodes[i2]) / 2, (nodes[i2] + nodes[i0]) / 2]
        kids += [(i0, m01, m20), (m01, i1, m12), (m20, m12, i2), (m01, m12, m20)]
        gk += [gj[j]] * 4
    nodes2 = np.concatenate([nodes, np.array(mids)])
    tris2 = np.array(kids)
    gk = np.array(gk)
    prob2 = direct.prepare(nodes, tris, np.concatenate([gj, gj, gj]), wl.grid, es_r_lo=wl.es_r_lo,
                           es_r_hi=wl.es_r_hi)
    prob2.g = np.concatenate([gk, gk, gk])
    a2 = iw.gridding_integrated(prob2, nodes2, tris2, 6, "kb", n=12)
    assert np.abs(a2 - a).max() <= 1e-10 * np.abs(a).max()


def test_integrated_near_field_pins():
    """The near-field values with the smooth kernel integrated over S_j: beyond
    the radius where the kept exponential sum matches 1/r to tol, a pair's
    value is at most tol times the exact integral of 1/r; and the complete
    route (integrated gridding plus this near field) meets the exact surface
    integrals of the element-constant density to the Fourier error, while the
    three-point route misses them by its quadrature error on this coarse
    sphere."""
    from oracle import nearfield as nfo
    from synth.workloads import sphere_random
    wl = sphere_random(2, 4, 64, 8)
    prob = direct.prepare_workload(wl)
    tol = 1e-3
    eps = nfo.near_radius(prob, tol, wl.es_r_hi)
    rp, cols, dist = nfo.near_pairs(wl.nodes, wl.tris, wl.nodes, 2.0 * eps)
    vals = iw.near_values_integrated(prob, wl.nodes, wl.tris, wl.nodes, rp, cols, n=12)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    exact_pair = nfo.triangle_potential(wl.nodes[rows], *(wl.nodes[wl.tris[cols, k]] for k in range(3)))
    far = dist >= eps
    assert far.sum() > 1000
    assert np.all(np.abs(vals[far]) <= tol * exact_pair[far])
    gbar = nfo.element_mean_density(prob, wl.tris.shape[0])
    exact = nfo.phi_exact_integrals(wl.nodes, wl.tris, gbar, wl.nodes)
    near_i, *_ = iw.phi_near_integrated(prob, wl.nodes, wl.tris, eps, n=12)
    comp_i = iw.phi_integrated(prob, wl.nodes, wl.tris, 8, "gauss", 12) + near_i
    near_3, *_ = nfo.phi_near(prob, wl.nodes, wl.tris, eps)
    comp_3 = direct.phi_ndft(prob) + near_3
    scale = np.abs(exact).max()
    assert np.abs(comp_i - exact).max() <= 2e-4 * scale
    assert np.abs(comp_3 - exact).max() >= 10 * np.abs(comp_i - exact).max()
