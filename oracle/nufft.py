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

The Kaiser-Bessel window of Sec. 3.2 (eq. KBfct, eq. cFB) is the alternative
(window="kb"): in grid units, psi(tau) = sinh(b sqrt(m^2 - tau^2)) /
(pi sqrt(m^2 - tau^2)) for |tau| <= m (value b / pi at |tau| = m), zero beyond
(the truncation to the cut-off m), b = pi (2 - 1/alpha); its 1-periodic Fourier
coefficients are psi^(l) = N^{-1} I_0(m sqrt(b^2 - (2 pi l / N)^2)) for
|l| <= N (1 - 1/(2 alpha)), which covers every kept mode |l| <= n/2.
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


def kb_shape(alpha):
    """b of the Kaiser-Bessel window (eq. KBfct)."""
    return np.pi * (2.0 - 1.0 / alpha)


def psi_kb(tau, m, b):
    """Kaiser-Bessel window in grid units, truncated to |tau| <= m (eq. KBfct)."""
    tau = np.asarray(tau, dtype=np.float64)
    s = np.sqrt(np.maximum(m * m - tau * tau, 0.0))
    safe = np.where(s > 0, s, 1.0)
    val = np.where(s > 0, np.sinh(b * s) / (np.pi * safe), b / np.pi)
    return np.where(np.abs(tau) <= m, val, 0.0)


def psi_hat_kb(l, N, m, b):
    """1-periodic Fourier coefficients of x -> psi_kb(N x) (eq. cFB)."""
    arg = b * b - (2.0 * np.pi * np.asarray(l, dtype=np.float64) / N) ** 2
    if np.any(arg < 0):
        raise ValueError("mode outside |l| <= N (1 - 1/(2 alpha))")
    return np.i0(m * np.sqrt(arg)) / N


class Window:
    """The window of Sec. 3.2 used by the gridding and the NFFT: "gauss"
    (default) or "kb"."""

    def __init__(self, m, alpha, kind="gauss"):
        if kind not in ("gauss", "kb"):
            raise ValueError(kind)
        self.m, self.alpha, self.kind = int(m), int(alpha), kind
        self.b = window_shape(m, alpha) if kind == "gauss" else kb_shape(alpha)

    def value(self, tau):
        if self.kind == "gauss":
            return psi(tau, self.b)
        return psi_kb(tau, self.m, self.b)

    def coeff(self, l, N):
        if self.kind == "gauss":
            return psi_hat(l, N, self.b)
        return psi_hat_kb(l, N, self.m, self.b)


def _stencil(t, win, N):
    """Per-axis stencil indices (mod N) and window values for points t [P]:
    returns idx [P, 2m], val [P, 2m]."""
    m = win.m
    f = np.floor(t)
    off = np.arange(-m + 1, m + 1, dtype=np.float64)
    r = f[:, None] + off[None, :]
    return np.mod(r, N).astype(np.int64), win.value(t[:, None] - r)


def _win(prob, m, window):
    return Window(m, prob.alpha, window)


def gridding(prob, m, window="gauss"):
    """Step 1: a_r on the oversampled grid (array [N1, N2, N3], real)."""
    N = [int(v) for v in prob.grid]
    win = _win(prob, m, window)
    t = prob.yt * np.asarray(N, dtype=np.float64)[None, :]
    ix, vx = _stencil(t[:, 0], win, N[0])
    iy, vy = _stencil(t[:, 1], win, N[1])
    iz, vz = _stencil(t[:, 2], win, N[2])
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


def spectrum_b(prob, a, m, window="gauss"):
    """Steps 2-3: b_l = c_l(f) / c_l(Upsilon~) for l in I_n ([n1, n2, n3],
    axis index l_q + n_q/2)."""
    N = [int(v) for v in prob.grid]
    win = _win(prob, m, window)
    A = np.fft.fftn(a) / float(np.prod(N))                  # c_l(f), eq. FFT
    sel = [np.mod(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    cf = A[np.ix_(sel[0], sel[1], sel[2])]
    den = [win.coeff(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    return cf / (den[0][:, None, None] * den[1][None, :, None] * den[2][None, None, :])


def nfft_grid(prob, d, m, window="gauss"):
    """Step 5a: g = IDFT(d / c(Upsilon~)) on I_{alpha n} (complex [N1, N2, N3])."""
    N = [int(v) for v in prob.grid]
    win = _win(prob, m, window)
    den = [win.coeff(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    gh = np.zeros(N, dtype=np.complex128)
    sel = [np.mod(_freq_index(int(prob.n[q])), N[q]) for q in range(3)]
    gh[np.ix_(sel[0], sel[1], sel[2])] = d / (den[0][:, None, None] * den[1][None, :, None]
                                             * den[2][None, None, :])
    return np.fft.ifftn(gh)


def interpolate(prob, g, m, targets=None, window="gauss"):
    """Step 5b: phi~_i = Re sum_r g_r Psi~(x~_i - r/N) over the 2m^3 stencil."""
    N = [int(v) for v in prob.grid]
    win = _win(prob, m, window)
    xt = prob.xt if targets is None else prob.xt[np.asarray(targets)]
    t = xt * np.asarray(N, dtype=np.float64)[None, :]
    ix, vx = _stencil(t[:, 0], win, N[0])
    iy, vy = _stencil(t[:, 1], win, N[1])
    iz, vz = _stencil(t[:, 2], win, N[2])
    gr = np.real(g)
    out = np.zeros(xt.shape[0])
    for i in range(2 * m):
        for j in range(2 * m):
            vals = gr[ix[:, i:i + 1], iy[:, j:j + 1], iz]          # [P, 2m]
            out += vx[:, i] * vy[:, j] * (vals * vz).sum(axis=1)
    return out


def phi_nufft(prob, m, targets=None, stages=False, window="gauss"):
    """phi_s at the nodes through steps 1-5; with stages=True also returns the
    intermediate arrays {a, b, d, g}."""
    a = gridding(prob, m, window)
    bl = spectrum_b(prob, a, m, window)
    cl = kernel.full_coefficients(prob.omega, prob.C, prob.n)
    d = cl * bl
    g = nfft_grid(prob, d, m, window)
    phi = interpolate(prob, g, m, targets, window) / FOUR_PI
    if stages:
        return phi, {"a": a, "b": bl, "d": d, "g": g}
    return phi
