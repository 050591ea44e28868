"""Pins of the reflecting-boundary oracle (cosine / sine transforms) against
results that do not come from its own formulas:
* the per-axis transforms equal scipy's DCT-III and DST-III (library
  routines) after the slot relabelling;
* the covariance equals the method-of-images sum of the periodic
  algorithms' exact covariance on the doubled grid (the periodic oracle,
  pinned elsewhere), for every family, several shapes and mixed axes;
* for a short Gaussian correlation the covariance equals the closed form
  C(x - x') +- C(x + x') (Neumann +, Dirichlet -) at every grid point."""
import itertools

import numpy as np
import pytest
from scipy import fft as sfft

from oracle import grf, noise, reflect, spectra


def _dct3(v):
    u = np.array(v, dtype=np.float64)
    u[1:] /= 2
    return sfft.dct(u, type=3)


def _dst3(v):
    n = len(v)
    u = np.empty(n)
    u[: n - 1] = np.asarray(v[1:], dtype=np.float64)[::-1] / 2
    u[n - 1] = v[0]
    return sfft.dst(u, type=3)


@pytest.mark.parametrize("n", [2, 4, 6, 10, 16, 30])
def test_axis_transforms_are_dct3_and_dst3(n):
    v = np.random.default_rng(n).normal(size=n)
    np.testing.assert_allclose(reflect.apply_basis(v, (False,)), _dct3(v), atol=1e-13)
    np.testing.assert_allclose(reflect.apply_basis(v, (True,)), _dst3(v), atol=1e-13)


@pytest.mark.parametrize("sine", list(itertools.product([False, True], repeat=3)), ids=str)
def test_separable_transform_3d(sine):
    dims = (4, 6, 8)
    v = np.random.default_rng(1).normal(size=dims)
    ref = v
    for ax, s in enumerate(sine):
        ref = np.apply_along_axis(_dst3 if s else _dct3, ax, ref)
    np.testing.assert_allclose(reflect.apply_basis(v, sine), ref, atol=1e-12)


def _image_sum(dims, lengths, sine, C2, jp):
    """sum over reflections r of s_r C2(j - r(jp)) on the N-grid."""
    dims = tuple(dims)
    out = np.zeros(dims)
    J = np.indices(dims)
    for r in itertools.product([0, 1], repeat=len(dims)):
        idx, sgn = [], 1.0
        for i, ri in enumerate(r):
            src = jp[i] if ri == 0 else -jp[i] - 1
            idx.append((J[i] - src) % (2 * dims[i]))
            if ri and sine[i]:
                sgn = -sgn
        out += sgn * C2[tuple(idx)]
    return out


FAMILIES = [
    dict(kind=spectra.MATERN, sigma=1.3, ell=0.2, nu=1.5),
    dict(kind=spectra.GAUSSIAN, sigma=0.7, ell=0.15),
    dict(kind=spectra.EXPONENTIAL, sigma=1.0, ell=0.3),
    dict(density=spectra.paper_density(5.0, 3, 1, 1), sigma=1.1),
]


@pytest.mark.parametrize("fam", range(len(FAMILIES)))
@pytest.mark.parametrize("dims,lengths", [((6,), (1.0,)), ((8, 6), (1.0, 0.8)), ((4, 6, 4), (0.5, 0.7, 0.6))], ids=str)
def test_covariance_is_the_image_sum_of_the_doubled_periodic_grid(fam, dims, lengths):
    f = FAMILIES[fam]
    dims2 = tuple(2 * n for n in dims)
    lengths2 = tuple(2 * l for l in lengths)
    if "density" in f:
        S2 = spectra.density_on_grid(dims2, lengths2, f["density"], half=False)
        C2 = grf.discrete_covariance(dims2, lengths2, None, 0, 0,
                                     h_full=spectra.filter_from_density(dims2, lengths2, S2, f["sigma"]))
    else:
        C2 = grf.discrete_covariance(dims2, lengths2, f["kind"], f["sigma"], f["ell"], f.get("nu", 0.5))
    rng = np.random.default_rng(len(dims))
    for sine in itertools.product([False, True], repeat=len(dims)):
        a = reflect.coefficients(dims, lengths, sine, **f)
        for _ in range(3):
            jp = tuple(int(rng.integers(n)) for n in dims)
            cov = reflect.covariance_with(a, sine, jp)
            ref = _image_sum(dims, lengths, sine, C2, jp)
            assert np.abs(cov - ref).max() <= 1e-12 * np.abs(C2).max(), (sine, jp)


@pytest.mark.parametrize("sine", [False, True])
def test_short_gaussian_correlation_matches_closed_form_images(sine):
    n, l, ell = 256, 1.0, 0.04
    a = reflect.coefficients((n,), (l,), (sine,), kind=spectra.GAUSSIAN, sigma=1.0, ell=ell)
    x = (np.arange(n) + 0.5) * l / n
    for jp in (0, 3, 17):
        cov = reflect.covariance_with(a, (sine,), (jp,))
        C = lambda r: spectra.covariance(spectra.GAUSSIAN, np.abs(r), 1.0, ell)
        ref = C(x - x[jp]) + (-1.0 if sine else 1.0) * C(x + x[jp])
        assert np.abs(cov - ref).max() <= 1e-10


def test_tabulated_and_density_coefficients_agree():
    dims, lengths, sine = (6, 8), (1.0, 2.0), (True, False)
    dens = spectra.paper_density(1.0, 1, 2, 1)
    S = dens(reflect.slot_components(dims, lengths, sine))
    S = np.broadcast_to(S, dims)
    np.testing.assert_array_equal(reflect.coefficients(dims, lengths, sine, S=S, sigma=2.0),
                                  reflect.coefficients(dims, lengths, sine, density=dens, sigma=2.0))


def test_sample_takes_the_contract_noise_with_its_own_tag():
    dims, lengths, sine = (4, 6), (1.0, 1.0), (False, True)
    a = reflect.coefficients(dims, lengths, sine, kind=spectra.MATERN, sigma=1.0, ell=0.3, nu=1.5)
    phi = reflect.sample(dims, lengths, sine, seed=7, batch=2, a=a)
    for b in range(2):
        z = noise.field_noise(dims, 7 + b, 2)
        np.testing.assert_array_equal(phi[b], reflect.field_from_noise(z, a, sine))
    assert not np.allclose(noise.field_noise(dims, 7, 2), noise.field_noise(dims, 7, 1))


# ---------------------------------------------------------------------------
# adjoint

@pytest.mark.parametrize("sine", [(False,), (True,), (False, True), (True, True, False)], ids=str)
def test_basis_transpose_identity(sine):
    dims = (6, 8, 4)[: len(sine)]
    rng = np.random.default_rng(len(sine))
    x, y = rng.normal(size=dims), rng.normal(size=dims)
    lhs = np.sum(reflect.apply_basis(x, sine) * y)
    rhs = np.sum(x * reflect.apply_basis_transpose(y, sine))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("kind,nu", [(spectra.MATERN, 1.5), (spectra.GAUSSIAN, 0.5), (spectra.EXPONENTIAL, 0.5)])
@pytest.mark.parametrize("dims,sine", [((8,), (True,)), ((6, 8), (False, True)), ((4, 6, 4), (True, False, True))],
                         ids=str)
def test_grad_theta_finite_differences(kind, nu, dims, sine):
    lengths = tuple(1.0 + 0.3 * i for i in range(len(dims)))
    z = noise.field_noise(dims, 3, 2)
    w = np.random.default_rng(0).uniform(size=dims)

    def loss(th):
        a = reflect.coefficients(dims, lengths, sine, kind=kind, sigma=th[0], ell=th[1], nu=th[2])
        return np.sum(w * reflect.field_from_noise(z, a, sine) ** 2)
    th = np.array([1.2, 0.3, nu])
    a = reflect.coefficients(dims, lengths, sine, kind=kind, sigma=th[0], ell=th[1], nu=th[2])
    g = 2 * w * reflect.field_from_noise(z, a, sine)
    got = reflect.grad_theta(z, g, lengths, sine, kind=kind, sigma=th[0], ell=th[1], nu=th[2])
    nparam = 3 if kind == spectra.MATERN else 2
    for i in range(nparam):
        e = np.zeros(3)
        e[i] = 1e-6 * th[i]
        fd = (loss(th + e) - loss(th - e)) / (2 * e[i])
        assert got[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    if nparam == 2:
        assert got[2] == 0.0


def test_grad_noise_finite_differences_and_density():
    dims, lengths, sine = (6, 8), (1.0, 2.0), (True, False)
    dens = spectra.paper_density(5.0, 3, 1, 1)
    a = reflect.coefficients(dims, lengths, sine, density=dens, sigma=1.3)
    z = noise.field_noise(dims, 1, 2)
    w = np.random.default_rng(1).uniform(size=dims)
    g = 2 * w * reflect.field_from_noise(z, a, sine)
    gz = reflect.grad_noise(g, a, sine)
    d = np.random.default_rng(2).normal(size=dims)
    loss = lambda zz: np.sum(w * reflect.field_from_noise(zz, a, sine) ** 2)
    fd = (loss(z + 1e-6 * d) - loss(z - 1e-6 * d)) / 2e-6
    assert np.sum(gz * d) == pytest.approx(fd, rel=1e-7)
    # a density-defined family: phi is linear in sigma, so sigma dL/dsigma = 2 L
    gt = reflect.grad_theta(z, g, lengths, sine, density=dens, sigma=1.3)
    assert gt[0] * 1.3 == pytest.approx(2 * loss(z), rel=1e-12)
    assert gt[1] == 0.0 and gt[2] == 0.0
