"""Smooth kernel N_s (exponential sum for 1/r) and its Fourier coefficients.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

SQRT_PI = np.sqrt(np.pi)


def expsum_sinc(h, r_lo, r_hi, tol):
    """Exponential sum 1/r ~ sum_t omega_t exp(-gamma_t r^2) (Sec. 3.3, eq. expsum).

    The paper takes a precomputed table from an external source; that table is
    not available, so the sum is built here from the integral representation
      1/r = (2/sqrt(pi)) int_R exp(-r^2 e^{2u} + u) du
    discretised by the trapezoidal rule with step h on nodes u_t = u_lo + t h,
    u_t <= u_hi:  omega_t = (2/sqrt(pi)) h e^{u_t},  gamma_t = e^{2 u_t}.
    u_hi = ln(7 / r_lo) drops upper terms below exp(-49) for r >= r_lo;
    u_lo = ln(tol sqrt(pi) / (2 r_hi)) drops a lower tail below tol relative
    for r <= r_hi. Physical units."""
    u_hi = np.log(7.0 / r_lo)
    u_lo = np.log(tol * SQRT_PI / (2.0 * r_hi))
    count = int(np.floor((u_hi - u_lo) / h)) + 1
    u = u_lo + h * np.arange(count, dtype=np.float64)
    omega = (2.0 / SQRT_PI) * h * np.exp(u)
    gamma = np.exp(2.0 * u)
    return omega, gamma


def truncate(omega, gamma, s, n, eta2):
    """Keep only the S' terms whose Fourier series on the torus is resolved by
    the grid (Sec. 3.3 'taking only S' <= S terms'; Sec. 5 eq. error_est3):
    in scaled units gamma_{t,q} = gamma_t / s_q^2, and term t is kept iff
    eta_{t,q}^2 = (pi n_q / 2)^2 / gamma_{t,q} >= eta2 on every axis q."""
    s = np.asarray(s, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    lim = (np.pi * n / 2.0) ** 2 / eta2                    # per axis
    gq = gamma[:, None] / (s[None, :] ** 2)                # [S, 3]
    keep = np.all(gq <= lim[None, :], axis=1)
    return omega[keep], gamma[keep]


def _gauss_legendre_panels(panels, order=16):
    """Composite Gauss-Legendre nodes/weights on [0, 1/2]."""
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 0.5, panels + 1)
    a, b = edges[:-1], edges[1:]
    half = 0.5 * (b - a)
    mid = 0.5 * (a + b)
    nodes = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    weights = (half[:, None] * w[None, :]).ravel()
    return nodes, weights


def fourier_coeff_1d(gamma_q, n):
    """c_{t,q}(l) = int_{-1/2}^{1/2} exp(-gamma_{t,q} xi^2) exp(-2 pi i l xi) dxi
    for l = 0..n/2 (eq. Fcoeff applied to one separable factor; the value is
    real and even in l). Composite Gauss-Legendre on [0, 1/2], doubled by
    symmetry. Returns [S', n/2 + 1]."""
    gamma_q = np.atleast_1d(np.asarray(gamma_q, dtype=np.float64))
    panels = max(n // 2 + 8, 16)
    xi, wq = _gauss_legendre_panels(panels)
    l = np.arange(n // 2 + 1, dtype=np.float64)
    cosm = np.cos(2.0 * np.pi * l[:, None] * xi[None, :])          # [L, P]
    f = np.exp(-gamma_q[:, None] * xi[None, :] ** 2)                # [S, P]
    return 2.0 * (f * wq[None, :]) @ cosm.T                          # [S, L]


def separable_coefficients(omega, gamma, s, n):
    """Per-axis factor tables C[q] = c_{t,q}(l), l = 0..n_q/2, with
    gamma_{t,q} = gamma_t / s_q^2 (Sec. 3.3: N_s and its Fourier series are sums
    of separable functions)."""
    return [fourier_coeff_1d(gamma / s[q] ** 2, int(n[q])) for q in range(3)]


def full_coefficients(omega, C, n):
    """c_l = sum_t omega_t prod_q c_{t,q}(|l_q|) for l in I_n
    (l_q = -n_q/2 .. n_q/2 - 1, axis order matches the returned array)."""
    idx = [np.abs(np.arange(-n[q] // 2, n[q] // 2)) for q in range(3)]
    A = [C[q][:, idx[q]] for q in range(3)]                          # [S, n_q]
    return np.einsum("t,ta,tb,tc->abc", omega, A[0], A[1], A[2], optimize=True)
