"""Pins of the oracle's density path for the covariance family of Section 4,
eq. (5), S(p) = (m^{kl} + (sum_i p_i^{2k})^l)^{-n}, and for tabulated
densities, against results that do not come from that formula:
* k = l = 1 is a Matern density (nu = n - d/2), pinned by its closed-form
  covariance elsewhere;
* k = 1, l = 2, n = 1 (d = 2) has the closed-form covariance
  C(r) = -(2 pi / m) kei(2 pi sqrt(m) r) (Kelvin function; C(0) = pi^2 / (2m));
* k >= 2, l = n = 1 (d = 2) has the variance
  (1/k^2) B(1/(2k), 1/(2k)) c^{1/k - 1} pi / sin(pi / k), c = m^k
  (Dirichlet integral), and the symmetries of the square but not of the
  circle (Figure 3(d) of the paper is the case m = 5, k = 3)."""
import numpy as np
import pytest
from scipy import special

from oracle import grf, spectra


def _cov(dims, lengths, density, sigma=1.0):
    S = spectra.density_on_grid(dims, lengths, density, half=False)
    h = spectra.filter_from_density(dims, lengths, S, sigma)
    return grf.discrete_covariance(dims, lengths, None, 1.0, 1.0, h_full=h)


@pytest.mark.parametrize("d,n", [(1, 1), (1, 2), (2, 2), (2, 3), (3, 2), (3, 4)])
@pytest.mark.parametrize("m", [0.75, 10.0])
def test_k_l_one_is_matern(d, n, m):
    nu = n - d / 2
    ell = np.sqrt(2 * nu / (4 * np.pi ** 2 * m))
    rng = np.random.default_rng(d * 10 + n)
    comps = [rng.normal(scale=3.0, size=200) for _ in range(d)]
    p2 = sum(c ** 2 for c in comps)
    fam = spectra.paper_density(m, 1, 1, n)(comps)
    mat = spectra.spectral_density(spectra.MATERN, p2, d, 1.0, ell, nu)
    zero = [np.zeros(1)] * d
    ratio = (fam / spectra.paper_density(m, 1, 1, n)(zero)) / (mat / spectra.spectral_density(spectra.MATERN, 0.0, d, 1.0, ell, nu))
    np.testing.assert_allclose(ratio, 1.0, rtol=1e-12)
    assert spectra.paper_density(m, 1, 1, n)(zero)[0] == pytest.approx(m ** (-n), rel=1e-15)


@pytest.mark.parametrize("m,L", [(0.75, 8.0), (10.0, 4.0)])
def test_k1_l2_kelvin_closed_form(m, L):
    """Figure 3(a)/(b) of the paper: m = 10 and 0.75, n = 1, k = 1, l = 2."""
    N = 512
    C = _cov((N, N), (L, L), spectra.paper_density(m, 1, 2, 1))
    closed = lambda r: -(2 * np.pi / m) * special.kei(2 * np.pi * np.sqrt(m) * r)
    c0 = np.pi ** 2 / (2 * m)
    assert closed(0.0) == pytest.approx(c0, rel=1e-12)
    r = np.arange(24) * L / N
    assert np.abs(C[0, :24] - closed(r)).max() <= 2e-3 * c0
    assert np.abs(C[:24, 0] - closed(r)).max() <= 2e-3 * c0
    i = np.arange(12)
    assert np.abs(C[i, i] - closed(np.sqrt(2) * i * L / N)).max() <= 2e-3 * c0


@pytest.mark.parametrize("k,m,N", [(2, 1.0, 1024), (3, 5.0, 512)])
def test_anisotropic_variance_and_symmetry(k, m, N):
    """(The grid truncates S at |p_i| = N / (2 L): its tail, ~N^(2-2k), bounds
    the tolerance.)"""
    L = 8.0
    C = _cov((N, N), (L, L), spectra.paper_density(m, k, 1, 1))
    c = m ** k
    var = (1 / k ** 2) * special.beta(1 / (2 * k), 1 / (2 * k)) * c ** (1 / k - 1) * np.pi / np.sin(np.pi / k)
    assert C[0, 0] == pytest.approx(var, rel=3e-4)
    np.testing.assert_allclose(C, C.T, atol=1e-15)                          # p1 <-> p2
    np.testing.assert_allclose(C, np.roll(C[::-1, :], 1, axis=0), atol=1e-15)   # x1 -> -x1
    # not rotation invariant: on the axis and on the diagonal at radius 1/4 the
    # covariances differ by more than 5% (axis index r N / L, diagonal r N / (L sqrt 2))
    ia, idg = int(round(0.25 * N / L)), int(round(0.25 * N / L / np.sqrt(2)))
    assert abs(C[0, ia] - C[idg, idg]) > 0.05 * abs(C[0, ia])


def test_tabulated_density_reproduces_its_family():
    """A tabulated S (here the Matern density on the grid) gives the filter of
    the family it tabulates; the sigma factor scales h."""
    dims, lengths = (24, 40), (1.5, 2.0)
    p2 = spectra.freq2_grid(dims, lengths, half=True)
    S = spectra.spectral_density(spectra.MATERN, p2, 2, 1.0, 0.2, 1.5)
    np.testing.assert_allclose(spectra.filter_from_density(dims, lengths, S, 2.0),
                               spectra.filter_h(dims, lengths, spectra.MATERN, 2.0, 0.2, 1.5), rtol=1e-14)


def test_sample_with_explicit_filter_equals_family_path():
    dims, lengths = (16, 20), (1.0, 1.3)
    h = spectra.filter_h(dims, lengths, spectra.GAUSSIAN, 1.0, 0.1, 0.5)
    for alg in (1, 2):
        a = grf.sample(dims, lengths, spectra.GAUSSIAN, 1.0, 0.1, seed=4, batch=2, alg=alg)
        b = grf.sample(dims, lengths, None, 0.0, 0.0, seed=4, batch=2, alg=alg, h=h)
        np.testing.assert_array_equal(a, b)
