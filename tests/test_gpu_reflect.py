"""GPU tests of reflecting boundaries (Neumann / Dirichlet by cosine / sine
transforms) against the float64 oracle: every axis mix in d = 1, 2, 3, both
precisions, every covariance family, tiles with a ragged tail, per-field
parameters, bit-for-bit invariance under batching, chunking and the noise
route, the covariance estimator, and host validation."""
import itertools
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import noise as onoise  # noqa: E402
from oracle import reflect  # noqa: E402
from oracle import spectra  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
NAMES = {False: "neumann", True: "dirichlet"}


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def bcs(sine):
    return tuple(NAMES[s] for s in sine)


def check(grf, dims, lengths, sine, dtype, seed=3, batch=2, **fam):
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, boundary=bcs(sine), **fam)
    phi = plan.sample(seed=seed, batch=batch).double().cpu().numpy()
    ofam = {k: v for k, v in fam.items()}
    if "cov" in ofam:
        ofam["kind"] = spectra.KIND_NAMES[ofam.pop("cov")]
    if "length_scale" in ofam:
        ofam["ell"] = ofam.pop("length_scale")
    ref = reflect.sample(dims, lengths, sine, seed=seed, batch=batch, **ofam)
    for b in range(batch):
        e = relerr(phi[b], ref[b])
        assert e <= TOL[dtype], (dims, sine, dtype, b, e)
    return plan, phi


MAT = dict(cov="matern", sigma=1.2, length_scale=0.15, nu=1.5)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims,lengths", [((8,), (1.0,)), ((64,), (2.0,)), ((1024,), (3.0,)),
                                          ((8, 24), (1.0, 1.5)), ((96, 128), (1.0, 1.2)),
                                          ((180, 64), (2.0, 1.0)), ((64, 1000), (0.5, 4.0)),
                                          ((16, 24, 32), (1.0, 1.5, 2.0)), ((12, 8, 24), (0.6, 0.4, 1.0))], ids=str)
def test_every_axis_mix_against_oracle(grf, dtype, dims, lengths):
    for sine in itertools.product([False, True], repeat=len(dims)):
        check(grf, dims, lengths, sine, dtype, **MAT)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("fam", [dict(cov="gaussian", sigma=0.8, length_scale=0.1),
                                 dict(cov="exponential", sigma=1.0, length_scale=0.3),
                                 dict(cov="matern", sigma=1.0, length_scale=0.05, nu=2.5)], ids=str)
@pytest.mark.parametrize("dims", [(256,), (128, 96), (24, 16, 48)], ids=str)
def test_families_against_oracle(grf, dtype, fam, dims):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    sine = tuple(i % 2 == 1 for i in range(len(dims)))
    check(grf, dims, lengths, sine, dtype, seed=11, **fam)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims", [(128,), (64, 96), (16, 12, 24)], ids=str)
def test_paper_family_and_tabulated(grf, dtype, dims):
    lengths = tuple(2.0 for _ in dims)
    sine = tuple(i == 0 for i in range(len(dims)))
    dens = spectra.paper_density(5.0, 3, 1, 1)
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, boundary=bcs(sine), cov="paper", sigma=1.3, m=5.0, k=3, l=1, n=1)
    phi = plan.sample(seed=5, batch=2).double().cpu().numpy()
    ref = reflect.sample(dims, lengths, sine, seed=5, batch=2, density=dens, sigma=1.3)
    assert relerr(phi, ref) <= TOL[dtype]
    S = np.broadcast_to(dens(reflect.slot_components(dims, lengths, sine)), dims)
    tab = grf.Plan(dims, lengths=lengths, dtype=dtype, boundary=bcs(sine), cov="tabulated", spectrum=S, sigma=1.3)
    phit = tab.sample(seed=5, batch=2).double().cpu().numpy()
    assert relerr(phit, ref) <= TOL[dtype]


@pytest.mark.parametrize("dims", [(512,), (32, 48), (8, 12, 16)], ids=str)
def test_per_field_parameters(grf, dims):
    """theta per field: the coefficients on the fly (no table)."""
    lengths = tuple(1.0 for _ in dims)
    sine = tuple(i % 2 == 0 for i in range(len(dims)))
    plan = grf.Plan(dims, lengths=lengths, dtype=torch.float64, boundary=bcs(sine), cov="matern")
    th = np.array([[1.0, 0.1, 1.5], [0.5, 0.3, 0.7], [2.0, 0.05, 3.0]])
    phi = plan.sample(seed=9, batch=3, theta=torch.tensor(th)).cpu().numpy()
    for b in range(3):
        ref = reflect.sample(dims, lengths, sine, seed=9 + b, batch=1, kind=spectra.MATERN,
                             sigma=th[b, 0], ell=th[b, 1], nu=th[b, 2])[0]
        assert relerr(phi[b], ref) <= 1e-12


@pytest.mark.parametrize("dims", [(2048,), (256, 256), (32, 32, 64)], ids=str)
def test_bitwise_invariance(grf, dims):
    """Same bits for a field whatever the batch, the chunking and the noise
    route (generated, or the same normals passed in)."""
    plan = grf.Plan(dims, boundary="dirichlet", **MAT)
    a = plan.sample(seed=100, batch=6)
    b = plan.sample(seed=103, batch=2)
    assert torch.equal(a[3:5], b)
    z = plan.noise(seed=100, batch=6)
    assert torch.equal(plan.sample_from_noise(z), a)
    zo = onoise.field_noise(dims, 101, 2)
    assert np.abs(z[1].double().cpu().numpy() - zo).max() <= 1e-5 * np.abs(zo).max()
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(int(np.prod(dims)) * 4 * 2 + 4)
    try:
        c = plan.sample(seed=100, batch=6)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(a, c)


@pytest.mark.parametrize("dims,sine", [((512, 512), (False, True)), ((64, 64, 64), (True, False, True))], ids=str)
def test_full_size_against_oracle(grf, dims, sine):
    check(grf, dims, tuple(1.0 for _ in dims), sine, torch.float32, seed=1, batch=2, **MAT)


@pytest.mark.parametrize("sine", [(False, False), (True, True), (True, False)], ids=str)
def test_statistical_covariance(grf, sine):
    """The covariance estimator on a reflecting plan: the estimate of
    Cov(phi_0, phi_x) matches the exact covariance (the oracle's) within its
    Monte Carlo error."""
    dims, lengths = (32, 48), (1.0, 1.5)
    plan = grf.Plan(dims, lengths=lengths, boundary=bcs(sine), **MAT)
    n = 20000
    est = plan.covariance(seed=0, nsamples=n).cpu().numpy()
    a = reflect.coefficients(dims, lengths, sine, kind=spectra.MATERN, sigma=1.2, ell=0.15, nu=1.5)
    c = reflect.covariance_with(a, sine, (0, 0))
    var = reflect.covariance_with(a, sine, (0, 0))[0, 0]
    vx = np.array([[reflect.covariance_with(a, sine, (i, j))[i, j] for j in range(dims[1])] for i in range(dims[0])])
    se = np.sqrt((var * vx + c ** 2) / n)
    assert np.all(np.abs(est - c) <= 6 * se), np.max(np.abs(est - c) / se)


def test_validation(grf):
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        grf.Plan((16, 16), boundary=("neumann", "periodic"))
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        grf.Plan((16, 16), alg=1, boundary="neumann")
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        grf.Plan((16, 16), boundary="neumann", draw_order="recursive")
    S = np.ones((16, 16))
    S[3, 4] = -1.0
    with pytest.raises(grf.GRFError, match="EINVAL"):
        grf.Plan((16, 16), boundary="neumann", cov="tabulated", spectrum=S)
    with pytest.raises(ValueError):
        grf.Plan((16, 16), boundary="neumann", cov="tabulated", spectrum=np.ones((16, 9)))
    with pytest.raises(KeyError):
        grf.Plan((16, 16), boundary="robin")


@pytest.mark.parametrize("sine", [False, True])
def test_statistical_covariance_1d(grf, sine):
    """d = 1: the estimator runs over sampled chunks (the fused 1D epilogue is
    the periodic sampler's)."""
    dims, lengths = (128,), (2.0,)
    plan = grf.Plan(dims, lengths=lengths, boundary=bcs((sine,)), **MAT)
    n = 100000
    est = plan.covariance(seed=1, nsamples=n).cpu().numpy()
    a = reflect.coefficients(dims, lengths, (sine,), kind=spectra.MATERN, sigma=1.2, ell=0.15, nu=1.5)
    c = reflect.covariance_with(a, (sine,), (0,))
    vx = np.array([reflect.covariance_with(a, (sine,), (i,))[i] for i in range(dims[0])])
    se = np.sqrt((c[0] * vx + c ** 2) / n)
    assert np.all(np.abs(est - c) <= 6 * se), np.max(np.abs(est - c) / se)
