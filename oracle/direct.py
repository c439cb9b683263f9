"""Direct evaluations of the single-layer potential (no window, no FFT).

Test infrastructure only (see oracle/__init__.py).

  R0  phi(x_i)   = 1/(4 pi) sum_k w_k g_k / |x_i - y_k|          (eq. slayer3 with
                   the three-point rule; the exact Newton kernel)
  R1  phi_s(x_i) = 1/(4 pi) sum_k w_k g_k K_F(x~_i - y~_k)        (eq. approx2, second
                   term, with N_s replaced by its Fourier series, eq. Fapprox)
  R2  phi_s(x_i) = 1/(4 pi) Re sum_{l in I_n} c_l b_l e^{2 pi i l.x~_i},
                   b_l = sum_k w_k g_k e^{-2 pi i l.y~_k}          (eq. smooth_phi with
                   b_l from eq. naive_gridding)

R1 and R2 are the same number by exchanging the order of summation
(eq. smooth_phi). The real part resolves the asymmetric index set
I_n = {-n/2 .. n/2-1}^3 (the potential is real).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry, kernel

FOUR_PI = 4.0 * np.pi


@dataclass
class Problem:
    """Everything the smooth-part definition needs, computed from the inputs."""
    y: np.ndarray        # quadrature points, physical [Mq, 3]
    w: np.ndarray        # quadrature weights [Mq]
    g: np.ndarray        # density at the quadrature points [Mq]
    x: np.ndarray        # targets (boundary nodes), physical [N, 3]
    c: np.ndarray        # scaling centre
    s: np.ndarray        # per-axis scale factors
    grid: np.ndarray     # oversampled grid N_q
    n: np.ndarray        # tensor grid n_q = N_q / alpha
    alpha: int
    omega: np.ndarray    # truncated exp-sum weights (S')
    gamma: np.ndarray    # truncated exp-sum exponents (S', physical units)
    C: list              # per-axis coefficient tables c_{t,q}(l), l = 0..n_q/2

    @property
    def q(self):
        return self.w * self.g

    @property
    def yt(self):
        return geometry.to_torus(self.y, self.c, self.s)

    @property
    def xt(self):
        return geometry.to_torus(self.x, self.c, self.s)


def prepare(nodes, tris, dens, grid, alpha=2, es_h=0.2, es_r_lo=None, es_r_hi=None,
            es_tol=1e-12, eta2=37.0, targets=None):
    """The problem instance. The potential is evaluated at the nodes, or at
    `targets` [P, 3] (e.g. all nodes of a volume mesh); the scaling always
    follows the body's nodes."""
    nodes = np.asarray(nodes, dtype=np.float64)
    grid = np.asarray(grid, dtype=np.int64)
    if np.any(grid % alpha) or np.any((grid // alpha) % 2):
        raise ValueError("grid must be alpha * n with n even")
    n = grid // alpha
    y, w = geometry.quadrature(nodes, tris)
    c, s = geometry.scaling(nodes, grid)
    om, ga = kernel.expsum_sinc(es_h, es_r_lo, es_r_hi, es_tol)
    om, ga = kernel.truncate(om, ga, s, n, eta2)
    C = kernel.separable_coefficients(om, ga, s, n)
    x = nodes if targets is None else np.asarray(targets, dtype=np.float64)
    return Problem(y=y, w=w, g=np.asarray(dens, dtype=np.float64), x=x, c=c, s=s,
                   grid=grid, n=n, alpha=int(alpha), omega=om, gamma=ga, C=C)


def prepare_workload(wl):
    return prepare(wl.nodes, wl.tris, wl.dens, wl.grid, wl.alpha, wl.es_h, wl.es_r_lo,
                   wl.es_r_hi, wl.es_tol, wl.eta2)


def _targets(prob, targets):
    if targets is None:
        return np.arange(prob.x.shape[0])
    return np.asarray(targets, dtype=np.int64)


def phi_exact_kernel(prob, targets=None, block=256):
    """R0: the three-point quadrature of the single layer potential with the
    exact Newton kernel 1/(4 pi |x - y|), physical units."""
    idx = _targets(prob, targets)
    q = prob.q
    out = np.empty(idx.shape[0])
    for a in range(0, idx.shape[0], block):
        xi = prob.x[idx[a:a + block]]
        d = np.sqrt(((xi[:, None, :] - prob.y[None, :, :]) ** 2).sum(-1))
        out[a:a + block] = (q[None, :] / d).sum(1) / FOUR_PI
    return out


def kernel_factor_1d(C, n, xi):
    """k_{t,q}(xi) = sum_{l=-n/2}^{n/2-1} c_{t,q}(l) e^{2 pi i l xi}
                  = c(0) + 2 sum_{l=1}^{n/2-1} c(l) cos(2 pi l xi) + c(n/2) e^{-i pi n xi}
    for every term t; xi [P] -> complex [P, S']."""
    h = n // 2
    l = np.arange(h, dtype=np.float64)
    fac = np.where(l == 0, 1.0, 2.0)
    cosm = fac[None, :] * np.cos(2.0 * np.pi * xi[:, None] * l[None, :])     # [P, h]
    real = cosm @ C[:, :h].T                                                 # [P, S']
    nyq = np.exp(-1j * np.pi * n * xi)[:, None] * C[None, :, h]
    return real + nyq


def fourier_kernel(prob, xi):
    """K_F(xi) = Re sum_t omega_t prod_q k_{t,q}(xi_q) for difference vectors
    xi [P, 3] in torus units."""
    k = [kernel_factor_1d(prob.C[q], int(prob.n[q]), xi[:, q]) for q in range(3)]
    return np.real((k[0] * k[1] * k[2]) @ prob.omega)


def phi_pairs(prob, targets=None, chunk=8192):
    """R1: O(M_q N) pair sum with the Fourier-series kernel K_F."""
    idx = _targets(prob, targets)
    q, yt, xt = prob.q, prob.yt, prob.xt
    out = np.zeros(idx.shape[0])
    for ii, i in enumerate(idx):
        acc = 0.0
        for a in range(0, yt.shape[0], chunk):
            xi = xt[i][None, :] - yt[a:a + chunk]
            acc += q[a:a + chunk] @ fourier_kernel(prob, xi)
        out[ii] = acc / FOUR_PI
    return out


def _phase(pts, n):
    """e^{-2 pi i l p} for l = -n/2 .. n/2-1, pts [P] -> [P, n]."""
    l = np.arange(-n // 2, n // 2, dtype=np.float64)
    return np.exp(-2j * np.pi * pts[:, None] * l[None, :])


def ndft_b(prob, chunk=None):
    """b_l = sum_k w_k g_k e^{-2 pi i l . y~_k} for l in I_n (eq. naive_gridding),
    as one matrix product per chunk of sources over (l_1) x (l_2, l_3)."""
    n1, n2, n3 = (int(v) for v in prob.n)
    yt, q = prob.yt, prob.q
    if chunk is None:
        chunk = max(256, int(2 ** 27 // (16 * n2 * n3)))
    b = np.zeros((n1, n2 * n3), dtype=np.complex128)
    for a in range(0, yt.shape[0], chunk):
        E1 = _phase(yt[a:a + chunk, 0], n1)
        E2 = _phase(yt[a:a + chunk, 1], n2)
        E3 = _phase(yt[a:a + chunk, 2], n3)
        KR = ((q[a:a + chunk, None] * E2)[:, :, None] * E3[:, None, :]).reshape(-1, n2 * n3)
        b += E1.T @ KR
    return b.reshape(n1, n2, n3)


def phi_ndft(prob, targets=None, b=None, chunk=None):
    """R2: phi_s(x_i) = 1/(4 pi) Re sum_{l in I_n} c_l b_l e^{2 pi i l . x~_i}."""
    idx = _targets(prob, targets)
    n1, n2, n3 = (int(v) for v in prob.n)
    if b is None:
        b = ndft_b(prob)
    cl = kernel.full_coefficients(prob.omega, prob.C, prob.n)
    d = (cl * b).reshape(n1, n2 * n3)
    xt = prob.xt[idx]
    if chunk is None:
        chunk = max(64, int(2 ** 27 // (16 * n2 * n3)))
    out = np.empty(idx.shape[0])
    for a in range(0, xt.shape[0], chunk):
        F1 = np.conj(_phase(xt[a:a + chunk, 0], n1))
        F2 = np.conj(_phase(xt[a:a + chunk, 1], n2))
        F3 = np.conj(_phase(xt[a:a + chunk, 2], n3))
        KR = (F2[:, :, None] * F3[:, None, :]).reshape(-1, n2 * n3)
        Y = KR @ d.T                                               # [P, n1]
        out[a:a + chunk] = np.real((F1 * Y).sum(axis=1)) / FOUR_PI
    return out
