"""Pins for oracle.kernel: exponential sum and Fourier coefficients (CPU only)."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import kernel


def test_expsum_approximates_inverse_distance():
    r_hi = np.sqrt(3.0)
    r_lo = 1e-3 * r_hi
    om, ga = kernel.expsum_sinc(0.2, r_lo, r_hi, 1e-12)
    r = np.geomspace(r_lo, r_hi, 10000)
    approx = (om[None, :] * np.exp(-ga[None, :] * r[:, None] ** 2)).sum(1)
    assert np.max(np.abs(r * approx - 1.0)) < 1e-10


def test_expsum_error_grows_with_step():
    # trapezoid error ~ 3 exp(-pi^2 / (2h)): a coarse step must be visibly worse
    r = np.geomspace(1e-2, 1.0, 2000)
    errs = []
    for h in (0.5, 0.35, 0.2):
        om, ga = kernel.expsum_sinc(h, 1e-2, 1.0, 1e-12)
        approx = (om[None, :] * np.exp(-ga[None, :] * r[:, None] ** 2)).sum(1)
        errs.append(np.max(np.abs(r * approx - 1.0)))
    assert errs[0] > 1e-5 and errs[1] > 1e-7 and errs[2] < 1e-10
    assert errs[0] > errs[1] > errs[2]


def _erf_closed_form(gamma, l):
    """int_{-1/2}^{1/2} e^{-g x^2} e^{-2 pi i l x} dx
    = sqrt(pi/g) e^{-pi^2 l^2/g} Re erf(sqrt(g)/2 + i pi l / sqrt(g))."""
    z = np.sqrt(gamma) / 2 + 1j * np.pi * l / np.sqrt(gamma)
    return np.sqrt(np.pi / gamma) * np.exp(-np.pi ** 2 * l ** 2 / gamma) * np.real(special.erf(z))


@pytest.mark.parametrize("gamma", [0.3, 1.0, 7.0, 40.0, 300.0, 2000.0])
def test_fourier_coeff_matches_erf(gamma):
    n = 64
    C = kernel.fourier_coeff_1d(np.array([gamma]), n)[0]
    for l in range(n // 2 + 1):
        if np.pi ** 2 * l ** 2 / gamma > 600:      # closed form overflows there
            continue
        ref = _erf_closed_form(gamma, l)
        assert abs(C[l] - ref) <= 1e-14 * max(1.0, abs(C[0])), (gamma, l, C[l], ref)


@pytest.mark.parametrize("gamma", [1e-20, 1e-6, 0.05, 5000.0])
def test_fourier_coeff_matches_adaptive_quadrature(gamma):
    n = 16
    C = kernel.fourier_coeff_1d(np.array([gamma]), n)[0]
    for l in range(n // 2 + 1):
        ref, _ = integrate.quad(lambda x: np.exp(-gamma * x * x) * np.cos(2 * np.pi * l * x),
                                -0.5, 0.5, limit=400, epsabs=1e-15, epsrel=1e-14)
        assert abs(C[l] - ref) < 1e-13, (gamma, l)


def test_fourier_coeff_limits():
    # gamma -> 0: the factor tends to 1 on the cell, so c(l) -> delta_{l0}
    C = kernel.fourier_coeff_1d(np.array([1e-30]), 32)[0]
    assert abs(C[0] - 1.0) < 1e-15 and np.max(np.abs(C[1:])) < 1e-15
    # large gamma: the whole-line transform sqrt(pi/g) exp(-pi^2 l^2 / g)
    g = 4000.0
    C = kernel.fourier_coeff_1d(np.array([g]), 128)[0]
    l = np.arange(65)
    ref = np.sqrt(np.pi / g) * np.exp(-np.pi ** 2 * l ** 2 / g)
    assert np.max(np.abs(C - ref)) < 1e-15


def test_truncation_rule():
    om = np.array([1.0, 2.0, 3.0, 4.0])
    ga = np.array([1.0, 10.0, 100.0, 1000.0])
    s = np.array([0.4, 0.4, 6.4])
    n = np.array([512, 512, 32])
    eta2 = 37.0
    # limit per axis (pi n/2)^2/eta2 on gamma/s^2: axis 0: 6.5e4*... compute by hand
    lim = (np.pi * n / 2) ** 2 / eta2
    keep = [all(g / s[q] ** 2 <= lim[q] for q in range(3)) for g in ga]
    o2, g2 = kernel.truncate(om, ga, s, n, eta2)
    assert list(g2) == [g for g, k in zip(ga, keep) if k]
    assert list(o2) == [o for o, k in zip(om, keep) if k]
    # gamma=1000: gamma/s_x^2 = 6250 <= (pi*256)^2/37 = 17484 kept; z: 1000/40.96=24.4 <= 68.3
    assert keep == [True, True, True, True]
    o3, g3 = kernel.truncate(om, ga, np.array([0.1, 0.4, 6.4]), n, eta2)
    assert list(g3) == [1.0, 10.0, 100.0]         # 1000/0.01 = 1e5 > 17484


def test_full_coefficients_against_3d_quadrature():
    """c_l of N_s(xi) = sum_t w_t prod_q exp(-g_t xi_q^2 / s_q^2) on the torus,
    by a direct 3-D tensor Gauss-Legendre quadrature (no separability used)."""
    om = np.array([0.7, 1.3])
    ga = np.array([0.5, 3.0])
    s = np.array([0.3, 0.5, 0.9])
    n = np.array([4, 6, 8])
    C = kernel.separable_coefficients(om, ga, s, n)
    full = kernel.full_coefficients(om, C, n)
    x, w = np.polynomial.legendre.leggauss(40)
    x, w = 0.5 * x, 0.5 * w                          # on [-1/2, 1/2]
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    f = sum(o * np.exp(-g * (X ** 2 / s[0] ** 2 + Y ** 2 / s[1] ** 2 + Z ** 2 / s[2] ** 2))
            for o, g in zip(om, ga))
    for l in [(0, 0, 0), (1, -2, 3), (-2, 2, -4), (-2, -3, 3), (1, 0, -1)]:
        e = np.exp(-2j * np.pi * (l[0] * X + l[1] * Y + l[2] * Z))
        ref = (W * f * e).sum()
        got = full[l[0] + n[0] // 2, l[1] + n[1] // 2, l[2] + n[2] // 2]
        assert abs(got - ref) < 1e-13 * abs(full).max(), l


def test_fourier_coeff_at_the_film_extremes():
    """The factor tables of the thin film (grid 1024 x 1024 x 64, n = 512, 512,
    32) at its largest kept exponents: along x (n = 512, gamma_{t,x} ~ 1.7e4,
    e^{-gamma/4} far below rounding) the coefficients equal the whole-line
    transform sqrt(pi/g) e^{-pi^2 l^2/g} for every l <= 256; along z (n = 32,
    gamma_{t,z} ~ 68, where the cell truncation still matters) they equal the
    erf closed form; both to 4e-15 of the peak, the rounding of the composite
    rule's sum over ~4000 points. This is the film's coefficient setup at its
    hardest terms."""
    from oracle import direct
    from synth.workloads import make_workload
    wl = make_workload("film512")
    p = direct.prepare_workload(wl)
    assert list(p.n) == [512, 512, 32]
    gx = p.gamma.max() / p.s[0] ** 2
    gz = p.gamma.max() / p.s[2] ** 2
    assert gx > 1e4 and 30 < gz < 100
    Cx = kernel.fourier_coeff_1d(np.array([gx]), 512)[0]
    l = np.arange(257)
    ref = np.sqrt(np.pi / gx) * np.exp(-np.pi ** 2 * l ** 2 / gx)
    assert np.max(np.abs(Cx - ref)) <= 4e-15 * ref[0]
    Cz = kernel.fourier_coeff_1d(np.array([gz]), 32)[0]
    for lz in range(17):
        assert abs(Cz[lz] - _erf_closed_form(gz, lz)) <= 1e-14 * Cz[0], lz
    # the table row the oracle builds for the film meets the same closed form
    assert np.max(np.abs(p.C[0][np.argmax(p.gamma)] - ref)) <= 4e-15 * ref[0]
