"""GPU tests of the adjoint of the reflecting-boundary sampler (Neumann /
Dirichlet) against the float64 oracle: parameter and noise gradients for
every axis mix in d = 1, 2, 3, both precisions, the families, per-field
parameters, the given-noise route and chunking (bit for bit)."""
import itertools
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import noise as onoise  # noqa: E402
from oracle import reflect  # noqa: E402
from oracle import spectra  # noqa: E402

NAMES = {False: "neumann", True: "dirichlet"}


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def bcs(sine):
    return tuple(NAMES[s] for s in sine)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims,lengths", [((8,), (1.0,)), ((64,), (2.0,)), ((1024,), (1.0,)), ((16, 24), (1.0, 1.5)),
                                          ((96, 128), (1.0, 1.0)), ((8, 12, 16), (1.0, 1.5, 2.0))], ids=str)
def test_every_axis_mix(grf, dtype, dims, lengths):
    params = (1.2, 0.15, 1.5)
    tol = 2e-5 if dtype == torch.float32 else 1e-10
    for sine in itertools.product([False, True], repeat=len(dims)):
        plan = grf.Plan(dims, lengths=lengths, dtype=dtype, boundary=bcs(sine), cov="matern", sigma=params[0],
                        length_scale=params[1], nu=params[2])
        B = 2
        phi = plan.sample(seed=5, batch=B).double().cpu().numpy()
        w = np.random.default_rng(1).uniform(size=(B,) + dims)
        g = 2 * w * phi
        gt, gz = plan.backward(torch.from_numpy(g), seed=5, need_noise_grad=True)
        gt, gz = gt.cpu().numpy(), gz.double().cpu().numpy()
        a = reflect.coefficients(dims, lengths, sine, kind=spectra.MATERN, sigma=params[0], ell=params[1], nu=params[2])
        for b in range(B):
            z = onoise.field_noise(dims, 5 + b, 2)
            ref = reflect.grad_theta(z, g[b], lengths, sine, kind=spectra.MATERN, sigma=params[0], ell=params[1],
                                     nu=params[2])
            assert np.abs(gt[b] - ref).max() <= tol * np.abs(ref).max(), (sine, b, gt[b], ref)
            rz = reflect.grad_noise(g[b], a, sine)
            assert np.abs(gz[b] - rz).max() <= tol * np.abs(rz).max(), (sine, b)


@pytest.mark.parametrize("cov,kind,params", [("gaussian", spectra.GAUSSIAN, (0.8, 0.1, 0.5)),
                                             ("exponential", spectra.EXPONENTIAL, (1.0, 0.3, 0.5))], ids=str)
@pytest.mark.parametrize("dims", [(256,), (64, 48), (16, 12, 24)], ids=str)
def test_families(grf, cov, kind, params, dims):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    sine = tuple(i % 2 == 1 for i in range(len(dims)))
    plan = grf.Plan(dims, lengths=lengths, dtype=torch.float64, boundary=bcs(sine), cov=cov, sigma=params[0],
                    length_scale=params[1], nu=params[2])
    phi = plan.sample(seed=2, batch=2).cpu().numpy()
    g = np.random.default_rng(3).normal(size=phi.shape) * phi
    gt, _ = plan.backward(torch.from_numpy(g), seed=2)
    gt = gt.cpu().numpy()
    for b in range(2):
        z = onoise.field_noise(dims, 2 + b, 2)
        ref = reflect.grad_theta(z, g[b], lengths, sine, kind=kind, sigma=params[0], ell=params[1], nu=params[2])
        assert np.abs(gt[b] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_per_field_routes_chunking_and_density(grf):
    dims, sine = (48, 64), (True, False)
    plan = grf.Plan(dims, dtype=torch.float64, boundary=bcs(sine), cov="matern")
    th = np.array([[1.0, 0.1, 1.5], [0.5, 0.3, 0.7], [2.0, 0.05, 3.0]])
    tt = torch.tensor(th)
    g = np.random.default_rng(2).normal(size=(3,) + dims)
    gt, gz = plan.backward(torch.from_numpy(g), seed=3, theta=tt, need_noise_grad=True)
    for b in range(3):
        z = onoise.field_noise(dims, 3 + b, 2)
        ref = reflect.grad_theta(z, g[b], (1.0, 1.0), sine, kind=spectra.MATERN, sigma=th[b, 0], ell=th[b, 1],
                                 nu=th[b, 2])
        assert np.abs(gt[b].cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    z = plan.noise(seed=3, batch=3)
    gt2, gz2 = plan.backward(torch.from_numpy(g), noise=z, theta=tt, need_noise_grad=True)
    assert torch.equal(gt, gt2) and torch.equal(gz, gz2)
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(48 * 64 * 8 + 8)
    try:
        gt3, gz3 = plan.backward(torch.from_numpy(g), seed=3, theta=tt, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(gt, gt3) and torch.equal(gz, gz3)
    # a family defined by its density: sigma dL/dsigma = 2 L, the rest 0
    pp = grf.Plan((32, 32, 16), lengths=(2.0, 2.0, 1.0), boundary="dirichlet", cov="paper", sigma=1.3, m=5.0, k=3, l=1,
                  n=1, dtype=torch.float64)
    phi = pp.sample(seed=8, batch=2)
    w = torch.rand(phi.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(phi.device)
    gtp, _ = pp.backward(2 * w * phi, seed=8)
    L = (w * phi ** 2).sum(dim=(1, 2, 3))
    np.testing.assert_allclose(gtp[:, 0].cpu().numpy() * 1.3, 2 * L.cpu().numpy(), rtol=1e-10)
    assert torch.all(gtp[:, 1:] == 0)
