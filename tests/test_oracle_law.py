"""Pins for the oracle's samplers: transforms against naive DFTs, realness,
Parseval, the exact covariance of the linear map, the config-1 statistical
test against the prescribed C(x), and the 1D convergence study of Section 4.
CPU only."""
import itertools

import numpy as np
import pytest

from oracle import dft, grf, noise, spectra

KINDS = [(spectra.GAUSSIAN, 1.0, 0.2, 0.5), (spectra.MATERN, 1.3, 0.3, 1.5),
         (spectra.EXPONENTIAL, 0.7, 0.25, 0.5), (spectra.MATERN, 1.0, 0.15, 2.5)]
SMALL = [((8,), (1.0,)), ((6, 4), (1.0, 1.0)), ((4, 10), (1.0, 2.5)), ((4, 6, 4), (1.0, 1.5, 0.5))]


def brute_cov(dims, lengths, kind, sigma, ell, nu):
    """(1/|D|) sum_k S(p_k) cos(2 pi p_k . x_j), p in the algorithms' centred
    order p_i = (k_i - N_i/2)/l_i, x_j = j_i l_i / N_i, summed term by term."""
    dims = tuple(dims)
    vol = float(np.prod(lengths))
    out = np.zeros(dims)
    for k in itertools.product(*[range(n) for n in dims]):
        p = np.array([(k[i] - dims[i] / 2) / lengths[i] for i in range(len(dims))])
        s = spectra.spectral_density(kind, np.sum(p ** 2), len(dims), sigma, ell, nu) / vol
        for j in itertools.product(*[range(n) for n in dims]):
            x = np.array([j[i] * lengths[i] / dims[i] for i in range(len(dims))])
            out[j] += s * np.cos(2 * np.pi * np.dot(p, x))
    return out


@pytest.mark.parametrize("dims,lengths", SMALL)
@pytest.mark.parametrize("alg", [1, 2])
def test_exact_covariance_of_linear_map(dims, lengths, alg):
    """phi = L z; Cov = L L^T must be the circulant of the discrete covariance."""
    kind, sigma, ell, nu = spectra.MATERN, 1.3, 0.3, 1.5
    f = grf.alg1_from_noise if alg == 1 else grf.alg2_from_noise
    P = int(np.prod(dims))
    L = np.zeros((P, P))
    for i in range(P):
        z = np.zeros(P)
        z[i] = 1
        L[:, i] = f(z.reshape(dims), lengths, kind, sigma, ell, nu).ravel()
    C = L @ L.T
    cn = brute_cov(dims, lengths, kind, sigma, ell, nu)
    idx = np.array(list(itertools.product(*[range(n) for n in dims])))
    for a in range(P):
        diff = (idx[a] - idx) % np.array(dims)
        ref = cn[tuple(diff.T)]
        np.testing.assert_allclose(C[a], ref, rtol=0, atol=1e-13 * cn.max())


@pytest.mark.parametrize("dims,lengths", SMALL)
def test_transforms_against_naive_dft(dims, lengths):
    rng = np.random.default_rng(5)
    z = rng.standard_normal(dims)
    kind, s, l, nu = KINDS[1]
    P = int(np.prod(dims))
    # one-FFT algorithm: phi = naive inverse DFT of the Hermitian-extended spectrum
    phi2, parts = grf.alg2_from_noise(z, lengths, kind, s, l, nu, return_parts=True)
    full = grf.hermitian_extend(parts["A"], dims)
    ref2 = dft.naive_dft(full, +1)
    assert np.abs(ref2.imag).max() <= 1e-13 * np.abs(ref2.real).max()
    np.testing.assert_allclose(phi2, ref2.real, atol=1e-13 * np.abs(phi2).max())
    # two-FFT algorithm: both transforms naive
    hfull = spectra.filter_h(dims, lengths, kind, s, l, nu, half=False)
    ref1 = dft.naive_dft(hfull * dft.naive_dft(z, -1) / np.sqrt(P), +1)
    phi1 = grf.alg1_from_noise(z, lengths, kind, s, l, nu)
    np.testing.assert_allclose(phi1, ref1.real, atol=1e-13 * np.abs(phi1).max())
    # naive DFT itself against a textbook case: a single plane wave
    k0 = tuple(1 % n for n in dims)
    e = np.zeros(dims, dtype=complex)
    e[k0] = 1
    wave = dft.naive_dft(e, +1)
    j = np.indices(dims)
    np.testing.assert_allclose(wave, np.exp(2j * np.pi * sum(j[i] * k0[i] / dims[i] for i in range(len(dims)))),
                               atol=1e-13)


@pytest.mark.parametrize("dims", [(16, 24), (8, 6, 10), (64,)])
def test_realness_and_c2r(dims):
    z = noise.field_noise(dims, 3, noise.TAG_ALG2)
    lengths = (1.0,) * len(dims)
    kind, s, l, nu = KINDS[0]
    full = grf.alg2_full_complex(z, lengths, kind, s, l, nu)
    phi = grf.alg2_from_noise(z, lengths, kind, s, l, nu)
    assert np.abs(full.imag).max() <= 1e-14 * np.abs(full.real).max()
    np.testing.assert_allclose(full.real, phi, atol=1e-14 * np.abs(phi).max())


@pytest.mark.parametrize("kindp", KINDS)
def test_parseval(kindp):
    dims = (12, 20)
    kind, s, l, nu = kindp
    z = noise.field_noise(dims, 9, noise.TAG_ALG2)
    phi, parts = grf.alg2_from_noise(z, (1.0, 1.0), kind, s, l, nu, return_parts=True)
    full = grf.hermitian_extend(parts["A"], dims)
    P = np.prod(dims)
    assert np.sum(phi ** 2) == pytest.approx(P * np.sum(np.abs(full) ** 2), rel=1e-12)


def test_alg1_equals_alg2_on_fourier_noise():
    """With xi := F[z]/sqrt(P) both algorithms compute the same field."""
    dims = (8, 12)
    z = noise.field_noise(dims, 4, noise.TAG_ALG1)
    kind, s, l, nu = KINDS[1]
    h = spectra.filter_h(dims, (1, 1), kind, s, l, nu)
    P = np.prod(dims)
    xi = np.fft.rfftn(z) / np.sqrt(P)
    # xi written through the naive DFT, then the one-FFT algorithm's inverse
    full = grf.hermitian_extend(h * xi, dims)
    phi2 = dft.naive_dft(full, +1).real
    np.testing.assert_allclose(grf.alg1_from_noise(z, (1, 1), kind, s, l, nu), phi2, atol=1e-13)


def test_config1_exact_and_statistical():
    """64 x 64 unit torus, Gaussian l = 0.05: the discrete covariance equals the
    prescribed C(x) to ~1e-20 (spectral mass beyond Nyquist ~1e-22, images
    e^-50), and the empirical covariance of the two-FFT sampler over 1024
    fields matches C within Monte Carlo error."""
    dims = (64, 64)
    kind, sigma, ell = spectra.GAUSSIAN, 1.0, 0.05
    cn = grf.discrete_covariance(dims, (1, 1), kind, sigma, ell)
    x = np.minimum(np.arange(64), 64 - np.arange(64)) / 64.0
    r = np.sqrt(x[:, None] ** 2 + x[None, :] ** 2)
    c = spectra.covariance(kind, r, sigma, ell)
    assert np.abs(cn - c).max() < 1e-14
    nf = 1024
    fields = grf.sample(dims, (1, 1), kind, sigma, ell, seed=0, batch=nf, alg=1)
    # covariance between every point and its lag-(a, b) neighbour, averaged
    lags = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 3), (5, 0), (0, 8), (32, 32)]
    for a, b in lags:
        prod = fields * np.roll(fields, shift=(-a, -b), axis=(1, 2))
        est = prod.mean()
        # standard error from the per-field means (fields independent)
        se = prod.mean(axis=(1, 2)).std(ddof=1) / np.sqrt(nf)
        assert abs(est - c[a, b]) < 5 * se + 1e-12, (a, b, est, c[a, b], se)


def test_one_dimensional_study_order():
    """Section 4's 1D example on [-pi, pi] (periodic grid of N points, l = 2 pi).
    Its density is the Matern one with nu = 7/2, ell = sqrt(0.07) (pinned in the
    spectra tests).  The sampler's exact covariance C_N against the closed form
    of Section 4 (summed over periodic images) shrinks at least like N^-4."""
    Cx = lambda x: (200 / 3 * np.abs(x) ** 3 + 40 * x ** 2 + 10 * np.abs(x) + 1) * np.exp(-10 * np.abs(x))
    assert Cx(0.0) == 1.0
    errs = []
    ns = list(range(2, 13))
    l = 2 * np.pi
    for n in ns:
        N = 2 ** n
        cn = grf.discrete_covariance((N,), (l,), spectra.MATERN, 1.0, np.sqrt(0.07), 3.5)
        x = np.arange(N) * l / N
        cper = sum(Cx(x + m * l) for m in range(-3, 4))
        errs.append(np.abs(cn - cper).max())
    errs = np.array(errs)
    slope = np.diff(np.log2(errs))          # per doubling of N
    # from N = 16 on (coarser grids do not resolve 1/ell) until rounding takes over
    assert np.all(slope[2:8] <= -4.0), slope
    assert errs[-1] < 1e-14
