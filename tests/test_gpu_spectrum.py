"""GPU tests of grf_debug_spectrum: the half-spectrum A = h xi that the
one-FFT sampler transforms (Section 3, the second algorithm: Philox noise,
Hermitian arrangement, filter), against the float64 oracle's A element by
element, and its documented packing (slot 0 = A(k, 0) + i A(k, N_d/2)),
checked by unpacking it with the mirrored rows and transforming it: the
result is the sampler's own field."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import grf as ogrf  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def _packed(A):
    """The oracle's half-spectrum [..., M + 1] in the library's packing."""
    M = A.shape[-1] - 1
    P = A[..., :M].copy()
    P[..., 0] = A[..., 0] + 1j * A[..., M]
    return P


def _unpack(Z):
    """[..., M] packed -> [..., M + 1]: A(k, 0) = (Z(k) + conj Z(-k)) / 2,
    A(k, M) = (Z(k) - conj Z(-k)) / (2i), -k over the leading axes."""
    lead = Z.shape[:-1]
    Zm = Z[..., 0]
    for ax in range(len(lead)):
        Zm = np.roll(np.flip(Zm, axis=ax), 1, axis=ax)
    A = np.concatenate([Z, np.zeros(lead + (1,), dtype=Z.dtype)], axis=-1)
    A[..., 0] = (Z[..., 0] + np.conj(Zm)) / 2
    A[..., -1] = (Z[..., 0] - np.conj(Zm)) / 2j
    return A


FAMILIES = [("matern", spectra.MATERN, (1.0, 0.1, 1.5)),
            ("gaussian", spectra.GAUSSIAN, (1.3, 0.07, 0.5)),
            ("exponential", spectra.EXPONENTIAL, (0.8, 0.05, 0.5))]
CASES = [((64, 96), (1.0, 1.5)), ((360, 64), (1.0, 1.0)), ((12, 8), (1.0, 1.0)), ((512, 512), (1.0, 1.0)),
         ((8, 12, 16), (1.0, 1.0, 1.0)), ((16, 24, 8), (2.0, 1.0, 1.0)), ((96,), (1.0,)), ((4096,), (2.0,))]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("cov,kind,params", FAMILIES, ids=str)
@pytest.mark.parametrize("dims,lengths", CASES, ids=str)
def test_spectrum_against_oracle(grf, dtype, cov, kind, params, dims, lengths):
    plan = grf.Plan(dims, lengths=lengths, alg=2, dtype=dtype, cov=cov, sigma=params[0], length_scale=params[1],
                    nu=params[2])
    B, seed = 2, 21
    Z = plan.spectrum(seed=seed, batch=B).to(torch.complex128).cpu().numpy()
    tol = 2e-6 if dtype == torch.float32 else 1e-13
    for b in range(B):
        z = onoise.field_noise(dims, seed + b, onoise.TAG_ALG2)
        _, parts = ogrf.alg2_from_noise(z, lengths, kind, *params, return_parts=True)
        ref = _packed(parts["A"])
        assert np.abs(Z[b] - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("dims", [(64, 96), (8, 12, 16), (360,)], ids=str)
def test_spectrum_transforms_to_the_sample(grf, dims):
    plan = grf.Plan(dims, alg=2, dtype=torch.float64, cov="matern")
    Z = plan.spectrum(seed=4, batch=2).cpu().numpy()
    phi = plan.sample(seed=4, batch=2).cpu().numpy()
    P = int(np.prod(dims))
    for b in range(2):
        ref = P * np.fft.irfftn(_unpack(Z[b]), s=dims, axes=tuple(range(len(dims))))
        assert np.abs(phi[b] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_spectrum_of_a_density_family(grf):
    dims, lengths = (64, 48), (2.0, 2.0)
    m, k, l, n, sigma = 0.75, 1, 2, 1, 1.2
    plan = grf.Plan(dims, lengths=lengths, alg=2, cov="paper", sigma=sigma, m=m, k=k, l=l, n=n, dtype=torch.float64)
    Z = plan.spectrum(seed=3, batch=1).cpu().numpy()[0]
    h = spectra.filter_from_density(dims, lengths, spectra.density_on_grid(dims, lengths, spectra.paper_density(m, k, l, n)),
                                    sigma)
    z = onoise.field_noise(dims, 3, onoise.TAG_ALG2)
    _, parts = ogrf.alg2_from_noise(z, lengths, spectra.MATERN, 1.0, 0.1, 1.5, return_parts=True, h=h)
    ref = _packed(parts["A"])
    assert np.abs(Z - ref).max() <= 1e-13 * np.abs(ref).max()


def test_spectrum_unsupported(grf):
    for kw in [dict(alg=1), dict(boundary="neumann"), dict(draw_order="recursive")]:
        plan = grf.Plan((32, 32), **kw)
        with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
            plan.spectrum(seed=0, batch=1)
