"""GPU tests of the recursive algorithm's draw order (Section 3): fields
sampled with draw_order='recursive' against the oracle's literal recursion
fed the same sequence, in d = 1, 2, 3 and both precisions, through both noise
routes, with batching/chunking invariance, the covariance estimator and host
validation."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import noise as onoise  # noqa: E402
from oracle import recursive  # noqa: E402
from oracle import spectra  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims,lengths", [((8,), (1.0,)), ((64,), (2.0,)), ((4096,), (1.0,)), ((4, 8), (1.0, 1.0)),
                                          ((96, 128), (1.0, 1.5)), ((180, 64), (2.0, 1.0)), ((64, 1000), (1.0, 2.0)),
                                          ((8, 12, 16), (1.0, 1.5, 2.0)), ((16, 24, 32), (1.0, 1.0, 1.0))], ids=str)
def test_against_literal_recursion(grf, dtype, dims, lengths):
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="matern", sigma=1.1, length_scale=0.2, nu=1.5,
                    draw_order="recursive")
    phi = plan.sample(seed=4, batch=2).double().cpu().numpy()
    ref = recursive.sample(dims, lengths, spectra.MATERN, 1.1, 0.2, 1.5, seed=4, batch=2)
    for b in range(2):
        assert relerr(phi[b], ref[b]) <= TOL[dtype], (dims, dtype, b, relerr(phi[b], ref[b]))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("dims", [(96, 128), (64, 1000), (16, 24, 32)], ids=str)
def test_per_field_theta(grf, dtype, dims):
    """Per-field (sigma, ell, nu): the generating pass evaluates h per entry
    instead of reading the plan's table; field b uses key seed + b."""
    lengths = (1.0,) * len(dims)
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="matern", draw_order="recursive")
    theta = np.array([[1.3, 0.15, 0.7], [0.8, 0.08, 2.2], [1.0, 0.3, 1.5]])
    phi = plan.sample(seed=7, batch=3, theta=torch.tensor(theta, device="cuda")).double().cpu().numpy()
    for b, (sg, ell, nu) in enumerate(theta):
        ref = recursive.sample(dims, lengths, spectra.MATERN, sg, ell, nu, seed=7 + b, batch=1)[0]
        assert relerr(phi[b], ref) <= TOL[dtype], (dims, dtype, b, relerr(phi[b], ref))


@pytest.mark.parametrize("dims", [(512, 512), (64, 64, 64)], ids=str)
def test_full_size(grf, dims):
    plan = grf.Plan(dims, cov="exponential", sigma=1.0, length_scale=0.05, draw_order="recursive")
    phi = plan.sample(seed=1, batch=1).double().cpu().numpy()
    ref = recursive.sample(dims, (1.0,) * len(dims), spectra.EXPONENTIAL, 1.0, 0.05, seed=1, batch=1)
    assert relerr(phi[0], ref[0]) <= 1e-5


def test_given_sequence_and_invariance(grf):
    """A sequence passed in (here random, not the Philox one) gives the
    literal recursion's field; the generated route equals the sequence route
    bit for bit; batching and chunking do not change a field."""
    dims = (48, 64)
    plan = grf.Plan(dims, dtype=torch.float64, cov="gaussian", sigma=1.0, length_scale=0.1, draw_order="recursive")
    z = np.random.default_rng(3).normal(size=(2,) + dims)
    phi = plan.sample_from_noise(torch.tensor(z)).cpu().numpy()
    for b in range(2):
        ref = recursive.alg3_from_stream(z[b].ravel(), dims, (1.0, 1.0), spectra.GAUSSIAN, 1.0, 0.1)
        assert relerr(phi[b], ref) <= 1e-12
    p32 = grf.Plan((256, 256), cov="matern", draw_order="recursive")
    a = p32.sample(seed=10, batch=6)
    assert torch.equal(p32.sample_from_noise(p32.noise(seed=10, batch=6)), a)
    assert torch.equal(p32.sample(seed=12, batch=3), a[2:5])
    zo = onoise.field_noise((256, 256), 11, 3)
    assert np.abs(p32.noise(seed=11, batch=1)[0].double().cpu().numpy() - zo).max() <= 1e-5 * np.abs(zo).max()
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(256 * 256 * 4 * 2 + 4)
    try:
        c = p32.sample(seed=10, batch=6)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(a, c)
    # another order of the same law: the counter order gives other fields
    assert not torch.equal(grf.Plan((256, 256), cov="matern").sample(seed=10, batch=1), a[:1])


def test_covariance_estimator_1d(grf):
    """The fused d = 1 estimator in the recursive order matches the exact
    covariance within its Monte Carlo error."""
    from oracle import grf as ogrf
    dims, l = (64,), (2.0,)
    plan = grf.Plan(dims, lengths=l, cov="matern", sigma=1.0, length_scale=0.3, nu=2.5, draw_order="recursive")
    n = 200000
    est = plan.covariance(seed=0, nsamples=n).cpu().numpy()
    C = ogrf.discrete_covariance(dims, l, spectra.MATERN, 1.0, 0.3, 2.5)
    se = np.sqrt((C[0] ** 2 + C ** 2) / n)
    assert np.all(np.abs(est - C) <= 6 * se)


def test_validation(grf):
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        grf.Plan((16, 16), alg=1, draw_order="recursive")
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        grf.Plan((16, 16), boundary="neumann", draw_order="recursive")
    with pytest.raises(KeyError):
        grf.Plan((16, 16), draw_order="sequential")
