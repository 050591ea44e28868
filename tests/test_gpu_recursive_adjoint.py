"""GPU tests of the adjoint in the recursive algorithm's draw order against
the float64 oracle: parameter gradients and the gradient with respect to the
sequence of draws, d = 1, 2, 3, both precisions, given and generated
sequences, chunking."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import noise as onoise  # noqa: E402
from oracle import recursive  # noqa: E402
from oracle import spectra  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims,lengths", [((8,), (1.0,)), ((1024,), (2.0,)), ((4, 8), (1.0, 1.0)),
                                          ((96, 128), (1.0, 1.5)), ((8, 12, 16), (1.0, 1.5, 2.0)),
                                          ((16, 16, 32), (1.0, 1.0, 1.0))], ids=str)
def test_against_oracle(grf, dtype, dims, lengths):
    params = (1.1, 0.2, 1.5)
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="matern", sigma=params[0], length_scale=params[1],
                    nu=params[2], draw_order="recursive")
    B = 2
    phi = plan.sample(seed=6, batch=B).double().cpu().numpy()
    w = np.random.default_rng(1).uniform(size=(B,) + dims)
    g = 2 * w * phi
    gt, gz = plan.backward(torch.from_numpy(g), seed=6, need_noise_grad=True)
    gt, gz = gt.cpu().numpy(), gz.double().cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-10
    for b in range(B):
        z = onoise.field_noise(dims, 6 + b, 3).ravel()
        ref = recursive.grad_theta(z, g[b], lengths, spectra.MATERN, *params)
        assert np.abs(gt[b] - ref).max() <= tol * np.abs(ref).max(), (b, gt[b], ref)
        rz = recursive.grad_stream(g[b], lengths, spectra.MATERN, *params)
        assert np.abs(gz[b] - rz).max() <= tol * np.abs(rz).max(), b


def test_routes_and_chunking(grf):
    dims = (64, 96)
    plan = grf.Plan(dims, cov="gaussian", length_scale=0.1, draw_order="recursive")
    g = torch.randn((5,) + dims, device="cuda", generator=torch.Generator(device="cuda").manual_seed(2))
    gt, gz = plan.backward(g, seed=9, need_noise_grad=True)
    z = plan.noise(seed=9, batch=5)
    gt2, gz2 = plan.backward(g, noise=z, need_noise_grad=True)
    assert torch.equal(gt, gt2) and torch.equal(gz, gz2)
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(64 * 96 * 4 * 2 + 4)
    try:
        gt3, gz3 = plan.backward(g, seed=9, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(gt, gt3) and torch.equal(gz, gz3)
