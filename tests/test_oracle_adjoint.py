"""Pins for the oracle's gradients: FP64 central finite differences (h = 1e-6),
the exact identities sigma dL/dsigma = 2L and z . grad_z L = 2L for the
quadratic loss L = sum w phi^2, and the brute-force transpose of the linear
map z -> phi.  CPU only."""
import numpy as np
import pytest

from oracle import adjoint, grf, noise, spectra

CASES = [(spectra.MATERN, 1.0, 0.1, 1.5), (spectra.GAUSSIAN, 1.2, 0.08, 0.5),
         (spectra.EXPONENTIAL, 0.9, 0.05, 0.5), (spectra.MATERN, 0.8, 0.2, 2.5)]
GRIDS = [((16, 24), (1.0, 1.0)), ((8, 6, 10), (1.0, 1.0, 2.0)), ((32,), (1.0,))]


def _loss(phi, w):
    return float(np.sum(w * phi * phi))


def _setup(dims, alg, seed=3):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0, 1, size=dims)
    z = noise.field_noise(dims, seed, noise.TAG_ALG2 if alg == 2 else noise.TAG_ALG1)
    return z, w


FWD = {1: grf.alg1_from_noise, 2: grf.alg2_from_noise}
GT = {1: adjoint.grad_theta_alg1, 2: adjoint.grad_theta_alg2}
GZ = {1: adjoint.grad_noise_alg1, 2: adjoint.grad_noise_alg2}


@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dims,lengths", GRIDS)
def test_theta_gradient_vs_central_differences(alg, case, dims, lengths):
    kind, sigma, ell, nu = case
    z, w = _setup(dims, alg)
    f = FWD[alg]
    phi = f(z, lengths, kind, sigma, ell, nu)
    g = 2 * w * phi
    got = GT[alg](z, g, lengths, kind, sigma, ell, nu)
    h = 1e-6
    th = [sigma, ell, nu]
    for i in range(3):
        if i == 2 and kind != spectra.MATERN:
            assert got[2] == 0.0
            continue
        tp, tm = list(th), list(th)
        tp[i] += h
        tm[i] -= h
        fd = (_loss(f(z, lengths, kind, *tp), w) - _loss(f(z, lengths, kind, *tm), w)) / (2 * h)
        assert got[i] == pytest.approx(fd, rel=2e-6, abs=1e-8 * abs(_loss(phi, w))), (i, got, fd)


@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("dims,lengths", GRIDS)
def test_homogeneity_identities(alg, dims, lengths):
    kind, sigma, ell, nu = CASES[0]
    z, w = _setup(dims, alg, seed=11)
    phi = FWD[alg](z, lengths, kind, sigma, ell, nu)
    L = _loss(phi, w)
    g = 2 * w * phi
    gt = GT[alg](z, g, lengths, kind, sigma, ell, nu)
    gz = GZ[alg](g, lengths, kind, sigma, ell, nu)
    assert sigma * gt[0] == pytest.approx(2 * L, rel=1e-12)
    assert float(np.sum(z * gz)) == pytest.approx(2 * L, rel=1e-12)


@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("dims", [(4, 6), (6, 4, 4), (8,), (2, 2)])
def test_noise_gradient_is_transpose_of_linear_map(alg, dims):
    kind, sigma, ell, nu = CASES[3]
    lengths = (1.0,) * len(dims)
    P = int(np.prod(dims))
    L = np.zeros((P, P))
    for i in range(P):
        e = np.zeros(P)
        e[i] = 1
        L[:, i] = FWD[alg](e.reshape(dims), lengths, kind, sigma, ell, nu).ravel()
    g = np.random.default_rng(2).standard_normal(P)
    got = GZ[alg](g.reshape(dims), lengths, kind, sigma, ell, nu).ravel()
    np.testing.assert_allclose(got, L.T @ g, atol=1e-13 * np.abs(L.T @ g).max())


def test_noise_gradient_spot_finite_differences():
    dims, lengths = (16, 24), (1.0, 1.0)
    kind, sigma, ell, nu = CASES[0]
    z, w = _setup(dims, 2, seed=5)
    phi = grf.alg2_from_noise(z, lengths, kind, sigma, ell, nu)
    gz = adjoint.grad_noise_alg2(2 * w * phi, lengths, kind, sigma, ell, nu)
    rng = np.random.default_rng(0)
    for _ in range(8):
        j = tuple(int(rng.integers(0, n)) for n in dims)
        for jj in [j, (j[0], 0), (j[0], 1), (0, 0), (8, 1)]:
            zp, zm = z.copy(), z.copy()
            zp[jj] += 1e-6
            zm[jj] -= 1e-6
            fd = (_loss(grf.alg2_from_noise(zp, lengths, kind, sigma, ell, nu), w)
                  - _loss(grf.alg2_from_noise(zm, lengths, kind, sigma, ell, nu), w)) / 2e-6
            assert gz[jj] == pytest.approx(fd, rel=1e-5, abs=1e-9)
