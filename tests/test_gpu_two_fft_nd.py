"""GPU tests of the two-FFT algorithm (Section 3, the first algorithm) in
d = 1 and d = 3 against the float64 oracle: the fields (white noise, forward
transform, filter h / sqrt(P) with the packed planes unpacked through the
mirrored row, inverse transform), the given-noise route and chunking (bitwise),
the launch sequence, the covariance estimator, and the adjoint (parameter
gradients from the two packed spectra F[g], F[z]; the noise gradient
F*[h F[g]] / sqrt(P))."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import grf as ogrf  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def _tol(dtype):
    return 1e-5 if dtype == torch.float32 else 1e-12


FAMILIES = [("matern", spectra.MATERN, (1.0, 0.1, 1.5)),
            ("gaussian", spectra.GAUSSIAN, (1.3, 0.07, 0.5)),
            ("exponential", spectra.EXPONENTIAL, (0.8, 0.05, 0.5))]

CASES = [((8,), (1.0,)), ((96,), (2.0,)), ((1000,), (1.0,)), ((4096,), (6.283185307179586,)),
         ((8, 12, 16), (1.0, 1.0, 1.0)), ((12, 4, 24), (1.0, 2.0, 1.0)), ((16, 24, 8), (1.5, 1.0, 1.0)),
         ((48, 32, 96), (1.0, 1.0, 1.0)), ((64, 64, 64), (1.0, 1.0, 1.0))]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("cov,kind,params", FAMILIES, ids=str)
@pytest.mark.parametrize("dims,lengths", CASES, ids=str)
def test_sample_against_oracle(grf, dtype, cov, kind, params, dims, lengths):
    plan = grf.Plan(dims, lengths=lengths, alg=1, dtype=dtype, cov=cov, sigma=params[0], length_scale=params[1],
                    nu=params[2])
    B, seed = 3, 11
    phi = plan.sample(seed=seed, batch=B).double().cpu().numpy()
    ref = ogrf.sample(dims, lengths, kind, *params, seed=seed, batch=B, alg=1)
    for b in range(B):
        err = np.abs(phi[b] - ref[b]).max() / np.abs(ref[b]).max()
        assert err <= _tol(dtype), (b, err)


@pytest.mark.parametrize("dims", [(360,), (24, 16, 32)], ids=str)
def test_routes_and_chunking_bitwise(grf, dims):
    plan = grf.Plan(dims, alg=1, dtype=torch.float32, cov="matern")
    B = 5
    a = plan.sample(seed=3, batch=B)
    z = plan.noise(seed=3, batch=B)
    assert torch.equal(plan.sample_from_noise(z), a)
    zo = onoise.batch_noise(dims, 3, B, onoise.TAG_ALG1)
    assert np.abs(z.double().cpu().numpy() - zo).max() <= 2e-5 * np.abs(zo).max()
    P = int(np.prod(dims))
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(2 * P * 4 + 4)
    try:
        c = plan.sample(seed=3, batch=B)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(a, c)
    one = torch.cat([plan.sample(seed=3 + b, batch=1) for b in range(B)])
    assert torch.equal(one, a)


def test_launch_sequence(grf):
    from paper_1105_2737_amd import _lib as L
    for dims, kinds in [((64,), [L.GRF_PASS_ROW_GEN_C2R]),
                        ((8, 12, 16), [L.GRF_PASS_ROW_R2C_GEN, L.GRF_PASS_COL_LOAD_FWD, 109,
                                       L.GRF_PASS_COL_LOAD_FWD, 110, L.GRF_PASS_COL_LOAD_INV,
                                       L.GRF_PASS_COL_LOAD_INV, L.GRF_PASS_ROW_C2R])]:
        plan = grf.Plan(dims, alg=1)
        assert [L.grf_sample_stage_info(plan.handle, 2, s)[0] for s in range(L.grf_sample_stage_count(plan.handle, 2))] \
            == kinds


def test_paper_family(grf):
    """A family given by its density (the filter is a table that holds the
    1/sqrt(P)); d = 3."""
    dims, lengths = (16, 12, 8), (1.0, 1.0, 2.0)
    m, k, l, n, sigma = 0.75, 1, 2, 1, 1.2
    plan = grf.Plan(dims, lengths=lengths, alg=1, cov="paper", sigma=sigma, m=m, k=k, l=l, n=n, dtype=torch.float64)
    phi = plan.sample(seed=2, batch=2).cpu().numpy()
    h = spectra.filter_from_density(dims, lengths, spectra.density_on_grid(dims, lengths, spectra.paper_density(m, k, l, n)),
                                    sigma)
    for b in range(2):
        z = onoise.field_noise(dims, 2 + b, onoise.TAG_ALG1)
        ref = ogrf.alg1_from_noise(z, lengths, spectra.MATERN, 1.0, 0.1, 1.5, h=h)
        assert np.abs(phi[b] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_covariance_estimator_d1(grf):
    """grf_covariance on a two-FFT d = 1 plan: (1/S) sum_s phi_s(0) phi_s(x),
    against the estimator formed from the same fields."""
    dims = (256,)
    plan = grf.Plan(dims, alg=1, dtype=torch.float64, cov="matern", length_scale=0.2)
    S = 64
    cov = plan.covariance(seed=7, nsamples=S).cpu().numpy()
    phi = plan.sample(seed=7, batch=S).cpu().numpy()
    ref = (phi[:, :1] * phi).mean(axis=0)
    assert np.abs(cov - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("cov,kind,params", FAMILIES, ids=str)
@pytest.mark.parametrize("dims,lengths", [((96,), (2.0,)), ((4096,), (1.0,)), ((8, 12, 16), (1.0, 1.0, 1.0)),
                                          ((12, 4, 24), (1.0, 2.0, 1.0)), ((48, 32, 96), (1.0, 1.0, 1.0))], ids=str)
def test_grad_theta_against_oracle(grf, dtype, cov, kind, params, dims, lengths):
    plan = grf.Plan(dims, lengths=lengths, alg=1, dtype=dtype, cov=cov, sigma=params[0], length_scale=params[1],
                    nu=params[2])
    B, seed = 2, 5
    w = np.random.default_rng(1).uniform(0, 1, size=(B,) + dims)
    phi = plan.sample(seed=seed, batch=B).double().cpu().numpy()
    g = 2 * w * phi
    gt, _ = plan.backward(torch.from_numpy(g), seed=seed)
    gt = gt.cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-10
    for b in range(B):
        z = onoise.field_noise(dims, seed + b, onoise.TAG_ALG1)
        ref = oadj.grad_theta_alg1(z, g[b], lengths, kind, *params)
        assert np.abs(gt[b] - ref).max() <= tol * np.abs(ref).max(), (b, gt[b], ref)
    L = (w * phi ** 2).reshape(B, -1).sum(axis=1)
    np.testing.assert_allclose(gt[:, 0] * params[0], 2 * L, rtol=tol * 10)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims", [(360,), (12, 16, 24)], ids=str)
def test_noise_gradient_and_routes(grf, dtype, dims):
    lengths = (1.0,) * len(dims)
    params = (1.2, 0.1, 2.5)
    plan = grf.Plan(dims, lengths=lengths, alg=1, dtype=dtype, cov="matern", sigma=params[0],
                    length_scale=params[1], nu=params[2])
    g = torch.randn((3,) + dims, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    gt, gz = plan.backward(g, seed=4, need_noise_grad=True)
    gzn = gz.double().cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-12
    for b in range(3):
        ref = oadj.grad_noise_alg1(g[b].numpy(), lengths, spectra.MATERN, *params)
        assert np.abs(gzn[b] - ref).max() <= tol * np.abs(ref).max()
    z = plan.noise(seed=4, batch=3)
    gt2, gz2 = plan.backward(g, noise=z, need_noise_grad=True)
    assert torch.equal(gt, gt2) and torch.equal(gz, gz2)
    P = int(np.prod(dims))
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(P * 8 + 8)
    try:
        gt3, gz3 = plan.backward(g, seed=4, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(gt, gt3) and torch.equal(gz, gz3)


@pytest.mark.parametrize("dims", [(512,), (16, 12, 24)], ids=str)
def test_per_field_parameters(grf, dims):
    """theta per field (sigma, ell, nu): the filter kernel reads field b's
    record; fields and parameter gradients against the oracle."""
    lengths = (1.0,) * len(dims)
    plan = grf.Plan(dims, alg=1, dtype=torch.float64, cov="matern")
    th = np.array([[1.0, 0.1, 1.5], [0.5, 0.3, 0.7], [2.0, 0.05, 3.0]])
    phi = plan.sample(seed=6, batch=3, theta=torch.tensor(th)).cpu().numpy()
    g = np.random.default_rng(4).normal(size=(3,) + dims)
    gt, _ = plan.backward(torch.from_numpy(g), seed=6, theta=torch.tensor(th))
    gt = gt.cpu().numpy()
    for b in range(3):
        z = onoise.field_noise(dims, 6 + b, onoise.TAG_ALG1)
        ref = ogrf.alg1_from_noise(z, lengths, spectra.MATERN, *th[b])
        assert np.abs(phi[b] - ref).max() <= 1e-12 * np.abs(ref).max()
        gref = oadj.grad_theta_alg1(z, g[b], lengths, spectra.MATERN, *th[b])
        assert np.abs(gt[b] - gref).max() <= 1e-10 * np.abs(gref).max()


@pytest.mark.parametrize("dims,alg", [((64,), 1), ((8, 12, 16), 1), ((64, 96), 1), ((64, 96), 2), ((4096,), 2)],
                         ids=str)
def test_empty_batch_everywhere(grf, dims, alg):
    """batch = 0 is a no-op for every entry point, whatever the output holds."""
    plan = grf.Plan(dims, alg=alg)
    out = torch.full((1,) + dims, 7.0, device="cuda")
    plan.sample(seed=0, batch=0, out=out)
    z = plan.noise(seed=0, batch=0)
    assert z.shape == (0,) + dims
    plan.sample_from_noise(z, out=out[:0])
    gt, gz = plan.backward(torch.zeros((0,) + dims), seed=0, need_noise_grad=True)
    assert gt.shape == (0, 3) and gz.shape == (0,) + dims
    if alg == 2:
        assert plan.spectrum(seed=0, batch=0).shape[0] == 0
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
