"""GPU tests of d = 1 sampling (Section 3 with a single row; the grids of the
one-dimensional study of Section 4) and of the statistical covariance
estimator of Section 4, against the float64 oracle."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import grf as ogrf  # noqa: E402
from oracle import spectra  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
KIND = {"gaussian": spectra.GAUSSIAN, "matern": spectra.MATERN, "exponential": spectra.EXPONENTIAL}
# Section 4's example: the Matern density with nu = 7/2, ell = sqrt(0.07) on [-pi, pi]
STUDY = dict(cov="matern", sigma=1.0, length_scale=float(np.sqrt(0.07)), nu=3.5)


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def with_env(env, fn):
    old = dict(os.environ)
    try:
        os.environ.update(env)
        return fn()
    finally:
        os.environ.clear()
        os.environ.update(old)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("N", [4, 8, 24, 64, 360, 1000, 1024, 2048, 4096])
def test_1d_against_oracle(grf, dtype, N):
    l = 2 * np.pi
    print("1d case:", N, dtype, flush=True)
    plan = grf.Plan((N,), lengths=(l,), alg=2, dtype=dtype, **STUDY)
    B = 5
    phi = plan.sample(seed=11, batch=B).double().cpu().numpy()
    ref = ogrf.sample((N,), (l,), spectra.MATERN, 1.0, STUDY["length_scale"], 3.5, seed=11, batch=B, alg=2)
    for b in range(B):
        assert relerr(phi[b], ref[b]) <= TOL[dtype], (N, b, relerr(phi[b], ref[b]))


@pytest.mark.parametrize("cov", ["gaussian", "exponential", "matern"])
def test_1d_covariance_families(grf, cov):
    N, l = 512, 3.0
    params = (1.3, 0.2, 2.5)
    plan = grf.Plan((N,), lengths=(l,), alg=2, dtype=torch.float64, cov=cov, sigma=params[0],
                    length_scale=params[1], nu=params[2])
    phi = plan.sample(seed=3, batch=4).cpu().numpy()
    ref = ogrf.sample((N,), (l,), KIND[cov], *params, seed=3, batch=4, alg=2)
    assert relerr(phi, ref) <= 1e-12


def test_1d_noise_theta_chunks(grf):
    """Supplied noise gives the generated bits; per-field theta matches plans
    with those parameters; cache-sized chunks (ragged) give the same bits."""
    N, B = 256, 9
    plan = grf.Plan((N,), alg=2, **STUDY)
    ref = plan.sample(seed=5, batch=B)
    z = plan.noise(seed=5, batch=B)
    assert torch.equal(plan.sample_from_noise(z), ref)
    got = with_env({"GRF_CHUNK_BYTES": str(4 * N * 4)}, lambda: plan.sample(seed=5, batch=B))
    assert torch.equal(got, ref)
    n = with_env({"GRF_CHUNK_BYTES": str(4 * N * 4)}, lambda: grf.grf_sample_stage_count(plan.handle, B))
    assert n == 3
    assert grf.grf_sample_stage_info(plan.handle, B, 0)[0] == grf.GRF_PASS_ROW_GEN_C2R
    theta = torch.tensor([[1.0, 0.1, 0.5], [2.0, 0.3, 1.5], [0.5, 0.05, 3.5]], dtype=torch.float64)
    per = plan.sample(seed=5, batch=3, theta=theta).double().cpu().numpy()
    for b in range(3):
        p1 = grf.Plan((N,), alg=2, cov="matern", sigma=float(theta[b, 0]), length_scale=float(theta[b, 1]),
                      nu=float(theta[b, 2]))
        one = p1.sample(seed=5 + b, batch=1)[0].double().cpu().numpy()
        assert relerr(per[b], one) <= 1e-6


def oracle_estimator(dims, lengths, params, seed, n):
    f = ogrf.sample(dims, lengths, spectra.MATERN, *params, seed=seed, batch=n, alg=2)
    flat = f.reshape(n, -1)
    return (flat[:, :1] * flat).mean(axis=0).reshape(dims)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dims,lengths,n,chunk", [((64,), (2 * np.pi,), 3000, None), ((4,), (2 * np.pi,), 5000, None),
                                                  ((2048,), (2 * np.pi,), 300, None),
                                                  ((32, 48), (1.0, 1.5), 700, 100 * 32 * 48 * 8)])
def test_covariance_matches_oracle_estimator(grf, dtype, dims, lengths, n, chunk):
    """The GPU estimator equals the oracle's (1/n) sum phi_b(0) phi_b(x) over
    the same fields (d = 1: the fused epilogue; d = 2: chunks, here several)."""
    params = (1.0, float(np.sqrt(0.07)), 3.5) if len(dims) == 1 else (1.0, 0.2, 1.5)
    plan = grf.Plan(dims, lengths=lengths, alg=2, dtype=dtype, cov="matern", sigma=params[0],
                    length_scale=params[1], nu=params[2])
    env = {} if chunk is None else {"GRF_CHUNK_BYTES": str(chunk)}
    got = with_env(env, lambda: plan.covariance(seed=7, nsamples=n)).cpu().numpy()
    ref = oracle_estimator(dims, lengths, params, 7, n)
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), np.abs(got - ref).max()


def test_covariance_converges_to_the_sampler_law(grf):
    """With many samples the estimate approaches the exact covariance of the
    sampled law C_N (oracle, closed form) within its Monte Carlo error: for
    Gaussian fields Var(phi(0) phi(x)) = C(0)^2 + C(x)^2."""
    N, l, n = 64, 2 * np.pi, 400000
    plan = grf.Plan((N,), lengths=(l,), alg=2, **STUDY)
    est = plan.covariance(seed=0, nsamples=n).cpu().numpy()
    cn = ogrf.discrete_covariance((N,), (l,), spectra.MATERN, 1.0, STUDY["length_scale"], 3.5)
    se = np.sqrt((cn[0] ** 2 + cn ** 2) / n)
    assert np.all(np.abs(est - cn) <= 6 * se), np.max(np.abs(est - cn) / se)
