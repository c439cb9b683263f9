"""R3: the smooth part through gridding, FFT, deconvolution and NFFT, step by step.

Test infrastructure only (see oracle/__init__.py). Follows Sec. 3 in order with
a Gaussian window (Sec. 3.2 names the Gaussian among the admissible windows):

  1. gridding   a_r = sum_k q_k Psi~(r/(alpha n) - y~_k)         (eq. gridding, with
                the quadrature sum of eq. naive_gridding in place of the
                triangle integrals)
  2. FFT        c_l(f) ~ |I_{alpha n}|^{-1} sum_r a_r e^{-2 pi i r.l/(alpha n)}  (eq. FFT)
  3. deconvolve b_l = c_l(f) / c_l(Upsilon~)                      (eq. deconv)
  4. multiply   d_l = c_l(N_s) b_l, l in I_n                       (Alg. 1)
  5. NFFT       phi_s(x_i) = Re sum_{l in I_n} d_l e^{2 pi i l.x~_i}, computed
                as the standard NFFT: g = IDFT(d / c(Upsilon~)) on I_{alpha n},
                then phi = sum_r g_r Psi~(x~_i - r/(alpha n))   (eq. convtheo)

Window (in grid units tau): psi(tau) = (pi b)^{-1/2} exp(-tau^2 / b),
b = 2 alpha m / ((2 alpha - 1) pi), truncated to the 2m grid points
floor(t) - m + 1 .. floor(t) + m around a point t (cut-off m, eq. wfct3 and
eq. indexset with the oversampled mesh size 1/(alpha n)), periodised (eq. wfct1).
Its 1-periodic Fourier coefficients are psi^(l) = N^{-1} exp(-b (pi l / N)^2).
Grid arrays are indexed [x, y, z] with r stored at r mod N.
"""
from __future__ import annotations

import numpy as np

from . import kernel

FOUR_PI = 4.0 * np.pi


def window_shape(m, alpha):
    return 2.0 * alpha * m / ((2.0 * alpha - 1.0) * np.pi)


def psi(tau, b):
    return np.exp(-tau * tau / b) / np.sqrt(np.pi * b)


def psi_hat(l, N, b):
    return np.exp(-b * (np.pi * l / N) ** 2) / N


def _stencil(t, m, b, N):
    """Per-axis stencil indices (mod N) and window values for points t [P]:
    returns idx [P, 2m], val [P, 2m]."""
    f = np.floor(t)
    off = np.arange(-m + 1, m + 1, dtype=np.float64)
    r = f[:, None] + off[None, :]
    return np.mod(r, N).astype(np.int64), psi(t[:, None] - r, b)


def gridding(prob, m):
    """Step 1: a_r on the oversampled grid (array [N1, N2, N3], real)."""
    N = [int(v) for v in prob.grid]
    b = window_shape(m, prob.alpha)
    t = prob.yt * np.asarray(N, dtype=np.float64)[None, :]
    ix, vx = _stencil(t[:, 0], m, b, N[0])
    iy, vy = _stencil(t[:, 1], m, b, N[1])
    iz, vz = _stencil(t[:, 2], m, b, N[2])
    q = prob.q
    a = np.zeros(N[0] * N[1] * N[2])
    for i in range(2 * m):
        for j in range(2 * m):
            flat = (ix[:, i:i + 1] * N[1] + iy[:, j:j + 1]) * N[2] + iz
            val = (q * vx[:, i] * vy[:, j])[:, None] * vz
            a += np.bincount(flat.ravel(), weights=val.ravel(), minlength=a.size)
    return a.reshape(N)


def _freq_index(n):
    return np.arange(-n // 2, n // 2)


def spectrum_b(prob, a, m):
    """Steps 2-3: b_l = c_l(f) / c_l(Upsilon~) for l in I_n ([n1, n2, n3],
    axis index l_q + n_q/2)."""
    N = [int(v) for v in prob.grid]
    b = window_shape(m, prob.alpha)
    A = np.fft.fftn(a) / float(np.prod(N))                  # c_l(f), eq. FFT
    sel = [np.mod(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    cf = A[np.ix_(sel[0], sel[1], sel[2])]
    den = [psi_hat(_freq_index(int(prob.n[q])), N[q], b) for q in range(3)]
    return cf / (den[0][:, None, None] * den[1][None, :, None] * den[2][None, None, :])


def nfft_grid(prob, d, m):
    """Step 5a: g = IDFT(d / c(Upsilon~)) on I_{alpha n} (complex [N1, N2, N3])."""
    N = [int(v) for v in prob.grid]
    b = window_shape(m, prob.alpha)
    den = [psi_hat(_freq_index(int(prob.n[q])), N[q], b) for q in range(3)]
    gh = np.zeros(N, dtype=np.complex128)
    sel = [np.mod(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    gh[np.ix_(sel[0], sel[1], sel[2])] = d / (den[0][:, None, None] * den[1][None, :, None]
                                             * den[2][None, None, :])
    return np.fft.ifftn(gh)


def interpolate(prob, g, m, targets=None):
    """Step 5b: phi~_i = Re sum_r g_r Psi~(x~_i - r/N) over the 2m^3 stencil."""
    N = [int(v) for v in prob.grid]
    b = window_shape(m, prob.alpha)
    xt = prob.xt if targets is None else prob.xt[np.asarray(targets)]
    t = xt * np.asarray(N, dtype=np.float64)[None, :]
    ix, vx = _stencil(t[:, 0], m, b, N[0])
    iy, vy = _stencil(t[:, 1], m, b, N[1])
    iz, vz = _stencil(t[:, 2], m, b, N[2])
    gr = np.real(g)
    out = np.zeros(xt.shape[0])
    for i in range(2 * m):
        for j in range(2 * m):
            vals = gr[ix[:, i:i + 1], iy[:, j:j + 1], iz]          # [P, 2m]
            out += vx[:, i] * vy[:, j] * (vals * vz).sum(axis=1)
    return out


def phi_nufft(prob, m, targets=None, stages=False):
    """phi_s at the nodes through steps 1-5; with stages=True also returns the
    intermediate arrays {a, b, d, g}."""
    a = gridding(prob, m)
    bl = spectrum_b(prob, a, m)
    cl = kernel.full_coefficients(prob.omega, prob.C, prob.n)
    d = cl * bl
    g = nfft_grid(prob, d, m)
    phi = interpolate(prob, g, m, targets) / FOUR_PI
    if stages:
        return phi, {"a": a, "b": bl, "d": d, "g": g}
    return phi
