"""Parity at the full benchmark configurations, in the launch layout the
benchmark times (the same plans and batch sizes, so the same cache-sized
chunks): sampled fields, including the first and last of each chunk, against
the float64 oracle."""
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


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("alg", [2, 1])
def test_512_squared_x1024(grf, alg):
    """Matern (1, 0.1, 1.5) on the unit torus, seeds 0..1023; 256 fields per
    chunk, so fields 255/256 and 511/512 sit on chunk boundaries."""
    plan = grf.Plan((512, 512), alg=alg, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    out = plan.sample(seed=0, batch=1024)
    for b in (0, 1, 255, 256, 511, 512, 1023):
        ref = ogrf.sample((512, 512), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5, seed=b, batch=1, alg=alg)[0]
        e = relerr(out[b].double().cpu().numpy(), ref)
        print(f"alg {alg} field {b}: {e:.3e}", flush=True)
        assert e <= 1e-5


def test_256_cubed_x16(grf):
    plan = grf.Plan((256, 256, 256), alg=2, dtype=torch.float32, cov="exponential", sigma=1.0, length_scale=0.05)
    out = plan.sample(seed=0, batch=16)
    for b in (0, 3, 4, 15):
        ref = ogrf.sample((256, 256, 256), (1.0, 1.0, 1.0), spectra.EXPONENTIAL, 1.0, 0.05, seed=b, batch=1, alg=2)[0]
        e = relerr(out[b].double().cpu().numpy(), ref)
        print(f"256^3 field {b}: {e:.3e}", flush=True)
        assert e <= 1e-5


def test_1024_squared_x64_forward_and_adjoint(grf):
    """The training configuration: L = sum w phi^2, w ~ U[0, 1]."""
    plan = grf.Plan((1024, 1024), alg=2, dtype=torch.float32, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    phi = plan.sample(seed=0, batch=64)
    w = torch.rand((64, 1024, 1024), device="cuda", generator=torch.Generator(device="cuda").manual_seed(1))
    g = 2 * w * phi
    gt, _ = plan.backward(g, seed=0)
    for b in (0, 63):
        ref = ogrf.sample((1024, 1024), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5, seed=b, batch=1, alg=2)[0]
        assert relerr(phi[b].double().cpu().numpy(), ref) <= 1e-5
        z = onoise.field_noise((1024, 1024), b, onoise.TAG_ALG2)
        rg = oadj.grad_theta_alg2(z, g[b].double().cpu().numpy(), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5)
        e = np.abs(gt[b].cpu().numpy() - rg).max() / np.abs(rg).max()
        print(f"1024^2 field {b}: grad rel err {e:.3e}", flush=True)
        assert e <= 2e-5
