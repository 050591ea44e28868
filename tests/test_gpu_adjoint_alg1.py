"""GPU tests of the adjoint of the two-FFT algorithm (d = 2) against the
float64 oracle: parameter gradients (xi = F[z] / sqrt(P) from the white
noise through the same transforms), the noise gradient F*[h F[g]] / sqrt(P),
per-field parameters, the given-noise route, chunking, and a family defined
by its density (its table holds the 1/sqrt(P))."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("cov,kind,params", [("matern", spectra.MATERN, (1.0, 0.1, 1.5)),
                                             ("gaussian", spectra.GAUSSIAN, (1.3, 0.07, 0.5)),
                                             ("exponential", spectra.EXPONENTIAL, (0.8, 0.2, 0.5))], ids=str)
@pytest.mark.parametrize("dims,lengths", [((64, 96), (1.0, 1.5)), ((360, 1000), (1.0, 1.0)), ((512, 512), (2.0, 2.0))],
                         ids=str)
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
    L = (w * phi ** 2).sum(axis=(1, 2))
    np.testing.assert_allclose(gt[:, 0] * params[0], 2 * L, rtol=tol * 10)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noise_gradient_and_routes(grf, dtype):
    dims, lengths, params = (96, 128), (1.0, 2.0), (1.2, 0.1, 2.5)
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
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(96 * 128 * 8 + 8)
    try:
        gt3, gz3 = plan.backward(g, seed=4, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(gt, gt3) and torch.equal(gz, gz3)


def test_per_field_parameters(grf):
    dims = (64, 64)
    plan = grf.Plan(dims, alg=1, dtype=torch.float64, cov="matern")
    th = np.array([[1.0, 0.1, 1.5], [0.5, 0.3, 0.7], [2.0, 0.05, 3.0]])
    tt = torch.tensor(th)
    g = np.random.default_rng(2).normal(size=(3,) + dims)
    gt, _ = plan.backward(torch.from_numpy(g), seed=3, theta=tt)
    gt = gt.cpu().numpy()
    for b in range(3):
        z = onoise.field_noise(dims, 3 + b, onoise.TAG_ALG1)
        ref = oadj.grad_theta_alg1(z, g[b], (1.0, 1.0), spectra.MATERN, *th[b])
        assert np.abs(gt[b] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_density_family(grf):
    dims, lengths, sigma = (64, 96), (2.0, 2.0), 1.3
    plan = grf.Plan(dims, lengths=lengths, alg=1, cov="paper", sigma=sigma, m=0.75, k=1, l=2, n=1, dtype=torch.float64)
    phi = plan.sample(seed=8, batch=2)
    w = torch.rand(phi.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(phi.device)
    gt, _ = plan.backward(2 * w * phi, seed=8)
    L = (w * phi ** 2).sum(dim=(1, 2))
    np.testing.assert_allclose(gt[:, 0].cpu().numpy() * sigma, 2 * L.cpu().numpy(), rtol=1e-10)
    assert torch.all(gt[:, 1:] == 0)
