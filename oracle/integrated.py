"""Integrated-window gridding: the paper's own type-1 step (Sec. 3.1, eq.
gridding and gridding2, the matrix A of eq. A), in which the window is
integrated over every triangle instead of being sampled at quadrature points
(eq. naive_gridding):

    a_r = sum_j g_j int_{S_j} Psi~(r / (alpha n) - y~) dsigma(y)

with the element density g_j (the mean of the three point values of a
density given at the quadrature points, as the near field takes it). The rest
of the route (FFT, deconvolution, multiplication by c_l(N_s), NFFT) is that of
`nufft`.

The integral over S_j is taken with the collapsed ("Duffy") tensor
Gauss-Legendre rule on the unit triangle: xi_1 = u (1 - v), xi_2 = u v with
Jacobian u, n Gauss points in u and in v, and dsigma = 2 |S_j| dxi. With that
rule the integrated gridding is exactly the point gridding of the n^2 mapped
points with weights 2 |S_j| w_u w_v u and charge g_j, so `nufft.gridding`
serves unchanged (its truncation of the window to -m < r - t <= m per axis is
the truncated window of eq. wfct3). `triangle_fourier` gives the closed form
of the integrated Fourier basis int_{S_j} exp(-2 pi i y~.l) dsigma (the
quantity the gridding approximates after deconvolution, eq. deconv) for the
pins. With integrated gridding the near-field correction (Sec. 3.4, eq.
nfcorr) subtracts the smooth kernel integrated over S_j by the same rule
(`near_values_integrated`), so that a near pair again carries the exact
integral of 1/r.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import geometry, kernel, nearfield, nufft


def duffy_rule(n):
    """Points (xi_1, xi_2) [n^2, 2] and weights [n^2] on the unit triangle
    (weights sum to 1/2)."""
    x, w = np.polynomial.legendre.leggauss(int(n))
    u, wu = 0.5 * (x + 1.0), 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    xi = np.stack([(U * (1.0 - V)).ravel(), (U * V).ravel()], axis=1)
    return xi, (WU * WV * U).ravel()


def triangle_points(nodes, tris, n):
    """Physical points [M, n^2, 3] and weights [M, n^2] of the rule on every
    triangle (weights sum to the triangle's area)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    P0, P1, P2 = (nodes[tris[:, k]] for k in range(3))
    xi, w = duffy_rule(n)
    pts = (P0[:, None, :] + xi[None, :, 0:1] * (P1 - P0)[:, None, :]
           + xi[None, :, 1:2] * (P2 - P0)[:, None, :])
    area = 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0), axis=1)
    return pts, 2.0 * area[:, None] * w[None, :]


def element_density(prob, M):
    """g_j = mean of the density at the three quadrature points of S_j."""
    g = np.asarray(prob.g, dtype=np.float64)
    return (g[:M] + g[M:2 * M] + g[2 * M:3 * M]) / 3.0


def gridding_integrated(prob, nodes, tris, m, window="gauss", n=12):
    """a_r of eq. gridding2 on the oversampled grid ([N1, N2, N3], real)."""
    M = tris.shape[0]
    pts, wts = triangle_points(nodes, tris, n)
    gj = element_density(prob, M)
    p = dataclasses.replace(prob, y=pts.reshape(-1, 3), w=wts.ravel(),
                            g=np.repeat(gj, pts.shape[1]))
    return nufft.gridding(p, m, window)


def phi_integrated(prob, nodes, tris, m, window="gauss", n=12, targets=None):
    """phi_s at the targets with integrated-window gridding (then eq. FFT,
    deconv, the multiplication by c_l(N_s) and the NFFT, as in `nufft`)."""
    a = gridding_integrated(prob, nodes, tris, m, window, n)
    bl = nufft.spectrum_b(prob, a, m, window)
    cl = kernel.full_coefficients(prob.omega, prob.C, prob.n)
    g = nufft.nfft_grid(prob, cl * bl, m, window)
    return nufft.interpolate(prob, g, m, targets, window) / nufft.FOUR_PI


def _e1(z):
    """(exp(z) - 1) / z, by its series for |z| < 1/2."""
    z = np.asarray(z, dtype=np.complex128)
    small = np.abs(z) < 0.5
    zs = np.where(small, z, 0.0)
    ser = np.zeros_like(z)
    term = np.ones_like(z)
    for k in range(1, 20):
        ser = ser + term
        term = term * zs / (k + 1)
    direct_ = (np.exp(z) - 1.0) / np.where(small, 1.0, z)
    return np.where(small, ser, direct_)


def _exp_dd2(x0, x1, x2):
    """Second divided difference of f(x) = exp(-i x) at real x0, x1, x2,
    evaluated stably: the two outermost points bound the difference quotient
    (f[a, b] = f(a) (-i) E1(-i (b - a))), and when all three lie within 1/2 of
    each other the Taylor series of f about x0 is used,
    f[x0, x1, x2] = f(x0) sum_k (-i)^(k+2) / (k+2)! sum_{p+q=k} d1^p d2^q."""
    X = np.stack([np.asarray(x0, float), np.asarray(x1, float), np.asarray(x2, float)])
    Xs = np.sort(X, axis=0)
    a, mid, b = Xs[0], Xs[1], Xs[2]
    D = b - a
    f = lambda x: np.exp(-1j * x)  # noqa: E731
    d_am = f(a) * (-1j) * _e1(-1j * (mid - a))
    d_mb = f(mid) * (-1j) * _e1(-1j * (b - mid))
    far = (d_mb - d_am) / np.where(D >= 0.5, D, 1.0)
    d1, d2 = mid - a, b - a
    ser = np.zeros(a.shape, dtype=np.complex128)
    hk = np.ones(a.shape)                       # sum_{p+q=k} d1^p d2^q
    p1 = np.ones(a.shape)                       # d1^k
    fact = 2.0
    for k in range(0, 25):
        ser = ser + (-1j) ** (k + 2) / fact * hk
        p1 = p1 * d1
        hk = hk * d2 + p1
        fact *= (k + 3)
    near = f(a) * ser
    return np.where(D >= 0.5, far, near)


def triangle_fourier(prob, nodes, tris, l):
    """int_{S_j} exp(-2 pi i y~ . l) dsigma(y) for every triangle [M]
    (complex). With theta_k = 2 pi y~_k . l at the vertices the integrand is
    exp(-i theta) of an affine theta, and by the Hermite-Genocchi formula the
    integral over the unit simplex of f''(lambda . theta) is the second divided
    difference f[theta_0, theta_1, theta_2]; with f(x) = -exp(-i x) (so that
    f'' = exp(-i x)) and dsigma = 2 |S_j| dxi the integral is
    -2 |S_j| exp(-i .)[theta_0, theta_1, theta_2]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    V = [geometry.to_torus(nodes[tris[:, k]], prob.c, prob.s) for k in range(3)]
    th = [2.0 * np.pi * (v @ l) for v in V]
    P0, P1, P2 = (nodes[tris[:, k]] for k in range(3))
    area = 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0), axis=1)
    return -2.0 * area * _exp_dd2(th[0], th[1], th[2])


def near_values_integrated(prob, nodes, tris, targets, rowptr, cols, n=12, chunk=20000):
    """C_ij = int_{S_j} dsigma / |x_i - y| - int_{S_j} N_s(|x_i - y|) dsigma for
    the pairs of a CSR pattern: the exact integral in closed form, the smooth
    kernel's by the collapsed rule with n x n points."""
    nodes = np.asarray(nodes, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    j = np.asarray(cols, dtype=np.int64)
    x = targets[rows]
    exact = nearfield.triangle_potential(x, nodes[tris[j, 0]], nodes[tris[j, 1]], nodes[tris[j, 2]])
    pts, wts = triangle_points(nodes, tris, n)
    smooth = np.zeros(j.size)
    for a in range(0, j.size, chunk):
        b = min(j.size, a + chunk)
        r = np.linalg.norm(x[a:b, None, :] - pts[j[a:b]], axis=2)
        smooth[a:b] = np.sum(wts[j[a:b]] * nearfield.smooth_kernel(prob, r), axis=1)
    return exact - smooth


def phi_near_integrated(prob, nodes, tris, eps, targets=None, n=12):
    """phi_NF at the targets with the values of `near_values_integrated` over
    the index sets of eq. nf_index. Returns (phi, rowptr, cols, vals)."""
    tg = nodes if targets is None else targets
    rowptr, cols, _ = nearfield.near_pairs(nodes, tris, tg, eps)
    vals = near_values_integrated(prob, nodes, tris, tg, rowptr, cols, n)
    gj = element_density(prob, tris.shape[0])
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    phi = np.bincount(rows, weights=vals * gj[cols], minlength=len(rowptr) - 1) / nufft.FOUR_PI
    return phi, rowptr, cols, vals
