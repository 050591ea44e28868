"""Pins for the spectral densities: normalisation, the closed-form
covariances they transform to, the paper's 1D example, and the analytic log
derivatives used by the adjoint.  CPU only."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import spectra

CASES = [(spectra.GAUSSIAN, 1.3, 0.1, 0.5), (spectra.MATERN, 1.0, 0.1, 1.5),
         (spectra.MATERN, 0.8, 0.05, 2.5), (spectra.MATERN, 1.0, 0.2, 0.5),
         (spectra.EXPONENTIAL, 1.1, 0.05, 0.5)]


def radial_transform(kind, sigma, ell, nu, d, r):
    """C(r) = int S(p) e^{-2 pi i p.x} dp for |x| = r, as a radial integral."""
    f = lambda p: spectra.spectral_density(kind, p * p, d, sigma, ell, nu)
    if d == 1:
        if r > 0:   # Fourier-weighted quadrature for the slowly decaying tail
            v, _ = integrate.quad(lambda p: 2 * f(p), 0, np.inf, weight="cos", wvar=2 * np.pi * r, limlst=200)
            return v
        g = lambda p: 2 * f(p)
    elif d == 2:
        g = lambda p: 2 * np.pi * p * f(p) * special.j0(2 * np.pi * p * r)
    else:
        g = lambda p: 4 * np.pi * p * p * f(p) * np.sinc(2 * p * r)
    v, _ = integrate.quad(g, 0, np.inf, limit=800, epsabs=1e-13, epsrel=1e-11)
    return v


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_density_transforms_to_covariance(case, d):
    kind, sigma, ell, nu = case
    if d == 3 and kind == spectra.EXPONENTIAL:
        pytest.skip("slowly decaying integrand; covered by the Matern nu=1/2 case")
    for r in [0.0, 0.5 * ell, 1.5 * ell]:
        got = radial_transform(kind, sigma, ell, nu, d, r)
        want = spectra.covariance(kind, r, sigma, ell, nu)
        # oscillatory quadrature of the heavy nu = 1/2 tails is good to ~1e-5
        assert got == pytest.approx(want, rel=2e-5, abs=2e-8), (d, r)


def test_exponential_is_matern_half():
    p2 = np.linspace(0, 50, 11)
    for d in (1, 2, 3):
        np.testing.assert_allclose(spectra.spectral_density(spectra.EXPONENTIAL, p2, d, 1.2, 0.07),
                                   spectra.spectral_density(spectra.MATERN, p2, d, 1.2, 0.07, 0.5), rtol=1e-14)
    r = np.linspace(0, 1, 9)
    np.testing.assert_allclose(spectra.covariance(spectra.MATERN, r, 1.2, 0.07, 0.5),
                               1.44 * np.exp(-r / 0.07), rtol=1e-12)


def test_paper_1d_example_is_matern_seven_halves():
    """Section 4: gamma(p) = 32e6/pi (100 + p^2)^-4 in the angular convention,
    variance 1, C(x) = (200/3|x|^3 + 40x^2 + 10|x| + 1) e^{-10|x|}.  In cycles,
    S(p) = 2 pi gamma(2 pi p); that is Matern with nu = 7/2, 2nu/ell^2 = 100."""
    p = np.linspace(0, 5, 21)
    paper = 2 * np.pi * 32e6 / np.pi * (100 + (2 * np.pi * p) ** 2) ** -4
    ours = spectra.spectral_density(spectra.MATERN, p ** 2, 1, 1.0, np.sqrt(0.07), 3.5)
    np.testing.assert_allclose(ours, paper, rtol=1e-12)
    x = np.linspace(0, 1.5, 16)
    closed = (200 / 3 * x ** 3 + 40 * x ** 2 + 10 * x + 1) * np.exp(-10 * x)
    np.testing.assert_allclose(spectra.covariance(spectra.MATERN, x, 1.0, np.sqrt(0.07), 3.5), closed, rtol=1e-10)
    # "the constant is used to scale the variance to 1"
    v, _ = integrate.quad(lambda q: 32e6 / np.pi * (100 + q * q) ** -4, -np.inf, np.inf)
    assert v == pytest.approx(1.0, rel=1e-10)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_log_derivatives_against_finite_differences(case, d):
    kind, sigma, ell, nu = case
    p2 = np.array([0.0, 3.0, 40.0, 900.0])
    ds, dl, dn = spectra.dlog_spectral_density(kind, p2, d, sigma, ell, nu)
    h = 1e-6
    logS = lambda s, l, n: np.log(spectra.spectral_density(kind, p2, d, s, l, n))
    fs = (logS(sigma + h, ell, nu) - logS(sigma - h, ell, nu)) / (2 * h)
    fl = (logS(sigma, ell + h * ell, nu) - logS(sigma, ell - h * ell, nu)) / (2 * h * ell)
    np.testing.assert_allclose(ds, fs, rtol=1e-7)
    np.testing.assert_allclose(dl, fl, rtol=1e-6, atol=1e-6)
    if kind == spectra.MATERN:
        fn = (logS(sigma, ell, nu + h) - logS(sigma, ell, nu - h)) / (2 * h)
        np.testing.assert_allclose(dn, fn, rtol=1e-6, atol=1e-7)
    else:
        assert np.all(dn == 0)


def test_wrapped_index():
    assert list(spectra.wrapped_index(6)) == [0, 1, 2, -3, -2, -1]
    np.testing.assert_array_equal(spectra.wrapped_index(8), np.fft.fftfreq(8, 1 / 8))
