"""Pins for oracle.nufft (R3): window, gridding normalisation, error decay in m."""
import numpy as np
import pytest
from scipy import integrate

from oracle import direct, nufft
from synth.workloads import sphere_random, make_workload


def test_window_integral_and_fourier_coefficients():
    for m in (2, 4, 8):
        b = nufft.window_shape(m, 2)
        L = 40.0 * np.sqrt(b)
        val, _ = integrate.quad(lambda t: nufft.psi(t, b), -L, L, points=[0.0], limit=200,
                                epsabs=1e-15, epsrel=1e-15)
        assert abs(val - 1.0) < 1e-12
        N = 64
        for l in (0, 3, 16):
            # coefficient of the periodised window x -> psi(N x) on [-1/2, 1/2)
            ref, _ = integrate.quad(lambda x: nufft.psi(N * x, b) * np.cos(2 * np.pi * l * x),
                                    -0.5, 0.5, points=[0.0], limit=200, epsabs=1e-16)
            assert abs(nufft.psi_hat(l, N, b) - ref) < 1e-14


def test_gridding_conserves_total_charge():
    """sum_r a_r = sum_k q_k prod_q sum_j psi(t - r_j); the inner sums equal 1
    up to truncation and aliasing (Poisson summation), so the total charge is
    reproduced to the window accuracy, increasingly so in m."""
    wl = sphere_random(2, 11, 32, 4)
    p = direct.prepare_workload(wl)
    qabs = np.abs(p.q).sum()
    errs = []
    for m in (2, 4, 6):
        a = nufft.gridding(p, m)
        errs.append(abs(a.sum() - p.q.sum()) / qabs)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-5


def test_b_tensor_error_decays_in_m():
    """Experiment of Sec. 3.2 (Fig. gridding_m) with the Gaussian window: the
    relative max-norm error of the computed tensor B against the exact
    quadrature sum of eq. naive_gridding decays geometrically in m."""
    wl = sphere_random(2, 7, 64, 2)        # n = 32, random g in place of m.n below
    p = direct.prepare_workload(wl)
    p.g = np.random.default_rng(7).uniform(-1, 1, size=p.g.size)
    exact = direct.ndft_b(p)
    errs = []
    for m in (2, 3, 4, 5, 6, 7):
        bl = nufft.spectrum_b(p, nufft.gridding(p, m), m)
        errs.append(np.abs(bl - exact).max() / np.abs(exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(r > 5 for r in ratios), errs
    # Gaussian bound ~ 4 exp(-pi m (1 - 1/(2 alpha - 1))) = 4 exp(-2 pi m / 3) at alpha = 2
    for m, e in zip((2, 3, 4, 5, 6, 7), errs):
        assert e < 4 * np.exp(-2 * np.pi * m / 3), (m, e)


def test_nufft_matches_definition_sphere_l3():
    """R3 against R2 (the definition) on the icosphere L3 / 64^3 workload:
    window error below 1e-6 from m = 6 on and decaying in m."""
    p = direct.prepare_workload(make_workload("sphere_l3"))
    ref = direct.phi_ndft(p)
    errs = {}
    for m in (4, 6, 8):
        phi = nufft.phi_nufft(p, m)
        errs[m] = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    assert errs[6] < 1e-6 and errs[8] < 1e-8 and errs[4] > errs[6] > errs[8]


def test_nufft_anisotropic_grid_and_alpha3():
    wl = sphere_random(1, 5, 24, 3)
    wl.grid = (24, 12, 36)
    wl.alpha = 3
    wl.grid = (24, 12, 36)                  # n = (8, 4, 12)
    p = direct.prepare_workload(wl)
    ref = direct.phi_pairs(p)
    phi = nufft.phi_nufft(p, 3)
    assert np.linalg.norm(phi - ref) < 2e-3 * np.linalg.norm(ref)


def _kb_bound(m, alpha=2):
    """Relative error bound of the NFFT with the Kaiser-Bessel window
    (eq. error_bound_nufft)."""
    return 4 * np.pi * (np.sqrt(m) + m) * (1 - 1 / alpha) ** 0.25 * np.exp(
        -2 * np.pi * m * np.sqrt(1 - 1 / alpha))


@pytest.mark.parametrize("m", [3, 4, 6])
def test_kb_fourier_pair(m):
    """eq. cFB against a numerical Fourier transform of eq. KBfct on the whole
    line: the inner part by adaptive quadrature, the oscillatory tail |tau| > m
    (sin branch) after tau = sqrt(u^2 + m^2) by QAWF with weight sin(b u)."""
    alpha, N = 2, 64
    b = nufft.kb_shape(alpha)
    for l in (0, 3, 11, N // 4):
        w = 2 * np.pi * l / N
        inner, _ = integrate.quad(lambda t: nufft.psi_kb(t, m, b) * np.cos(w * t), 0, m,
                                  limit=200, epsabs=0, epsrel=1e-13)
        tail, _ = integrate.quad(
            lambda u: np.cos(w * np.sqrt(u * u + m * m)) / (np.pi * np.sqrt(u * u + m * m)),
            0, np.inf, weight="sin", wvar=b, limlst=200)
        ft = 2 * (inner + tail)
        assert abs(ft - N * nufft.psi_hat_kb(l, N, m, b)) <= 1e-9 * ft, (m, l)


def test_kb_window_values():
    m, b = 4, nufft.kb_shape(2)
    tau = np.array([-m - 0.5, -m, -1.0, 0.0, 2.5, m])
    v = nufft.psi_kb(tau, m, b)
    assert v[0] == 0.0
    assert np.isclose(v[1], b / np.pi) and np.isclose(v[5], b / np.pi)
    assert np.isclose(v[3], np.sinh(b * m) / (np.pi * m))
    assert np.isclose(v[2], np.sinh(b * np.sqrt(15.0)) / (np.pi * np.sqrt(15.0)))


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_kb_composite_error_within_bound(m):
    """R3 with the Kaiser-Bessel window against the definition (R2) on the
    icosphere L3: within the univariate bound of eq. error_bound_nufft, and far
    below the Gaussian's error at the same m."""
    wl = make_workload("sphere_l3", m)
    p = direct.prepare_workload(wl)
    ref = direct.phi_ndft(p)
    e_kb = np.linalg.norm(nufft.phi_nufft(p, m, window="kb") - ref) / np.linalg.norm(ref)
    e_g = np.linalg.norm(nufft.phi_nufft(p, m) - ref) / np.linalg.norm(ref)
    assert e_kb <= _kb_bound(m)
    assert e_kb < 0.1 * e_g
