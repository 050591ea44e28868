"""GPU tests of the adjoint of the one-FFT sampler in d = 1 and d = 3 (the
d = 2 case is in test_gpu_parity.py) against the float64 oracle: parameter
gradients for every family, per-field parameters, the noise gradient (with
the 3D planes k_d = 0, N_d/2 unpacked from Z(k) and Z(-k)), invariance under
chunking, and the family of Section 4 through its table."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402

FAMS = [("matern", spectra.MATERN, (1.0, 0.1, 1.5)), ("gaussian", spectra.GAUSSIAN, (1.3, 0.07, 0.5)),
        ("exponential", spectra.EXPONENTIAL, (0.8, 0.2, 0.5))]


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("fam", range(3), ids=[f[0] for f in FAMS])
@pytest.mark.parametrize("dims,lengths", [((64,), (1.0,)), ((4096,), (2.0,)), ((16, 24, 32), (1.0, 1.5, 2.0)),
                                          ((32, 32, 64), (1.0, 1.0, 1.0))], ids=str)
def test_grad_theta_against_oracle(grf, dtype, fam, dims, lengths):
    name, kind, params = FAMS[fam]
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov=name, sigma=params[0], length_scale=params[1], nu=params[2])
    B, seed = 2, 7
    w = np.random.default_rng(1).uniform(0, 1, size=(B,) + dims)
    phi = plan.sample(seed=seed, batch=B).double().cpu().numpy()
    g = 2 * w * phi
    gt, _ = plan.backward(torch.from_numpy(g), seed=seed)
    gt = gt.cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-10
    for b in range(B):
        z = onoise.field_noise(dims, seed + b, onoise.TAG_ALG2)
        ref = oadj.grad_theta_alg2(z, g[b], lengths, kind, *params)
        assert np.abs(gt[b] - ref).max() <= tol * np.abs(ref).max(), (b, gt[b], ref)
    # sigma dL/dsigma = 2 L (phi is linear in sigma)
    L = (w * phi ** 2).sum(axis=tuple(range(1, len(dims) + 1)))
    np.testing.assert_allclose(gt[:, 0] * params[0], 2 * L, rtol=tol * 10)


@pytest.mark.parametrize("dims", [(512,), (8, 12, 16)], ids=str)
def test_per_field_parameters(grf, dims):
    lengths = (1.0,) * len(dims)
    plan = grf.Plan(dims, dtype=torch.float64, cov="matern")
    th = np.array([[1.0, 0.1, 1.5], [0.5, 0.3, 0.7], [2.0, 0.05, 3.0]])
    tt = torch.tensor(th)
    phi = plan.sample(seed=3, batch=3, theta=tt).cpu().numpy()
    g = np.random.default_rng(2).normal(size=phi.shape)
    gt, _ = plan.backward(torch.from_numpy(g), seed=3, theta=tt)
    gt = gt.cpu().numpy()
    for b in range(3):
        z = onoise.field_noise(dims, 3 + b, onoise.TAG_ALG2)
        ref = oadj.grad_theta_alg2(z, g[b], lengths, spectra.MATERN, *th[b])
        assert np.abs(gt[b] - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims", [(64,), (2048,), (8, 12, 16), (16, 16, 16), (4, 8, 8)], ids=str)
def test_noise_gradient_against_oracle(grf, dtype, dims):
    lengths = tuple(1.0 + 0.5 * i for i in range(len(dims)))
    params = (1.2, 0.1, 2.5)
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="matern", sigma=params[0], length_scale=params[1],
                    nu=params[2])
    z = plan.noise(seed=2, batch=2)
    g = torch.randn((2,) + dims, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    gt, gz = plan.backward(g, noise=z, need_noise_grad=True)
    gz = gz.double().cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-12
    for b in range(2):
        ref = oadj.grad_noise_alg2(g[b].numpy(), lengths, spectra.MATERN, *params)
        assert np.abs(gz[b] - ref).max() <= tol * np.abs(ref).max()
    # the generated noise and the same noise passed in give the same gradients
    gt2, gz2 = plan.backward(g, seed=2, need_noise_grad=True)
    assert torch.equal(gt, gt2) and np.array_equal(gz, gz2.double().cpu().numpy())


@pytest.mark.parametrize("dims", [(4096,), (64, 64, 64)], ids=str)
def test_chunking_keeps_bits(grf, dims):
    plan = grf.Plan(dims, cov="matern")
    B = 6
    g = torch.randn((B,) + dims, device="cuda", generator=torch.Generator(device="cuda").manual_seed(4))
    ref_t, ref_z = plan.backward(g, seed=1, need_noise_grad=True)
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(int(np.prod(dims)) * 4 * 2 + 8)   # 2 fields per chunk
    try:
        t2, z2 = plan.backward(g, seed=1, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(ref_t, t2) and torch.equal(ref_z, z2)


def test_paper_family_3d(grf):
    """Table-only family: dL/dsigma from linearity, the other derivatives 0."""
    dims, lengths, sigma = (16, 24, 32), (2.0, 2.0, 2.0), 1.4
    plan = grf.Plan(dims, lengths=lengths, cov="paper", sigma=sigma, m=5.0, k=3, l=1, n=1, dtype=torch.float64)
    phi = plan.sample(seed=8, batch=2)
    w = torch.rand(phi.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(phi.device)
    gt, _ = plan.backward(2 * w * phi, seed=8)
    L = (w * phi ** 2).sum(dim=(1, 2, 3))
    np.testing.assert_allclose(gt[:, 0].cpu().numpy() * sigma, 2 * L.cpu().numpy(), rtol=1e-10)
    assert torch.all(gt[:, 1:] == 0)


def test_autograd_3d(grf):
    dims = (16, 16, 32)
    plan = grf.Plan(dims, dtype=torch.float32, cov="matern")
    theta = torch.tensor([[1.0, 0.1, 1.5]] * 2, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.rand((2,) + dims, device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    phi = grf.GRFSample.apply(theta, plan, 3)
    (w * phi.double() ** 2).sum().backward()
    Lb = (w * phi.double() ** 2).sum(dim=(1, 2, 3))
    np.testing.assert_allclose(theta.grad[:, 0].cpu().numpy(), (2 * Lb / theta[:, 0]).detach().cpu().numpy(),
                               rtol=1e-5)
