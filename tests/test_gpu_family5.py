"""GPU tests of the covariance family of Section 4, eq. (5), and of tabulated
densities: sampling (d = 1, 2, 3; both algorithms in 2D), the adjoint's noise
gradient and sigma derivative, the statistical covariance of Figure 3's
method, and host validation -- against the float64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import grf as ogrf  # noqa: E402
from oracle import spectra  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
# Figure 3 of the paper (a)-(d), and two of Figure 4's densities
FIG = [(10.0, 1, 2, 1), (0.75, 1, 2, 1), (10.0, 1, 1, 3), (5.0, 3, 1, 1), (1.0, 1, 1, 2), (1.0, 2, 1, 1)]


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def oracle_h(dims, lengths, mkln, sigma=1.0):
    S = spectra.density_on_grid(dims, lengths, spectra.paper_density(*mkln), half=True)
    return spectra.filter_from_density(dims, lengths, S, sigma)


def paper_plan(grf, dims, lengths, mkln, dtype=torch.float32, alg=2, sigma=1.0):
    m, k, l, n = mkln
    return grf.Plan(dims, lengths=lengths, alg=alg, dtype=dtype, cov="paper", sigma=sigma, m=m, k=k, l=l, n=n)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("mkln", FIG, ids=str)
def test_paper_family_2d_against_oracle(grf, dtype, mkln):
    dims, lengths = (96, 128), (2.0, 2.5)
    plan = paper_plan(grf, dims, lengths, mkln, dtype, sigma=1.5)
    phi = plan.sample(seed=21, batch=3).double().cpu().numpy()
    ref = ogrf.sample(dims, lengths, None, 0, 0, seed=21, batch=3, alg=2, h=oracle_h(dims, lengths, mkln, 1.5))
    for b in range(3):
        assert relerr(phi[b], ref[b]) <= TOL[dtype], (mkln, b, relerr(phi[b], ref[b]))


@pytest.mark.parametrize("dims,lengths,alg", [((64,), (3.0,), 2), ((1024,), (6.0,), 2), ((16, 24, 32), (1.0, 1.5, 2.0), 2),
                                              ((64, 96), (1.0, 1.0), 1), ((512, 512), (4.0, 4.0), 2)])
def test_paper_family_other_shapes(grf, dims, lengths, alg):
    mkln = (5.0, 3, 1, 1)
    for dtype in (torch.float32, torch.float64):
        plan = paper_plan(grf, dims, lengths, mkln, dtype, alg=alg)
        phi = plan.sample(seed=2, batch=2).double().cpu().numpy()
        ref = ogrf.sample(dims, lengths, None, 0, 0, seed=2, batch=2, alg=alg, h=oracle_h(dims, lengths, mkln))
        assert relerr(phi, ref) <= TOL[dtype], (dims, alg, dtype, relerr(phi, ref))


def test_tabulated_density(grf):
    """A tabulated Matern density reproduces the oracle's Matern fields; a
    tabulated family (5) density reproduces the family's plan."""
    dims, lengths = (128, 96), (1.0, 1.2)
    p2 = spectra.freq2_grid(dims, lengths, half=True)
    S = spectra.spectral_density(spectra.MATERN, p2, 2, 1.0, 0.1, 1.5)
    for dtype in (torch.float32, torch.float64):
        tab = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="tabulated", spectrum=S, sigma=2.0)
        phi = tab.sample(seed=4, batch=2).double().cpu().numpy()
        ref = ogrf.sample(dims, lengths, spectra.MATERN, 2.0, 0.1, 1.5, seed=4, batch=2, alg=2)
        assert relerr(phi, ref) <= TOL[dtype]
    Sp = spectra.density_on_grid(dims, lengths, spectra.paper_density(5.0, 3, 1, 1), half=True)
    a = grf.Plan(dims, lengths=lengths, cov="tabulated", spectrum=Sp).sample(seed=9, batch=2)
    b = paper_plan(grf, dims, lengths, (5.0, 3, 1, 1)).sample(seed=9, batch=2)
    assert relerr(a.double().cpu().numpy(), b.double().cpu().numpy()) <= 1e-6


def test_tabulated_validation_and_theta(grf):
    dims = (32, 48)
    S = np.ones((32, 25))
    S[1, 0] = 2.0                                     # breaks S(p) = S(-p) on the plane k_d = 0
    with pytest.raises(grf.GRFError, match="EINVAL"):
        grf.Plan(dims, cov="tabulated", spectrum=S)
    S[1, 0] = 1.0
    S[5, 3] = -1.0
    with pytest.raises(grf.GRFError, match="EINVAL"):
        grf.Plan(dims, cov="tabulated", spectrum=S)
    plan = paper_plan(grf, dims, (1.0, 1.0), (1.0, 1, 1, 2))
    with pytest.raises(grf.GRFError, match="EUNSUPPORTED"):
        plan.sample(seed=0, batch=2, theta=torch.tensor([1.0, 0.1, 1.5], dtype=torch.float64))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_paper_family_adjoint(grf, dtype):
    """dL/dz against the oracle; dL/dsigma from phi being linear in sigma
    (sigma dL/dsigma = 2 L for L = sum w phi^2); the other parameters do not
    exist for this family (derivative 0)."""
    dims, lengths, mkln, sigma = (64, 96), (2.0, 2.0), (0.75, 1, 2, 1), 1.3
    plan = paper_plan(grf, dims, lengths, mkln, dtype, sigma=sigma)
    B = 2
    w = torch.rand((B,) + dims, generator=torch.Generator().manual_seed(0), dtype=torch.float64)
    phi = plan.sample(seed=8, batch=B)
    g = (2 * w.to(phi.device) * phi.double()).to(dtype)
    gt, gz = plan.backward(g, seed=8, need_noise_grad=True)
    h = oracle_h(dims, lengths, mkln, sigma)
    tol = 1e-5 if dtype == torch.float32 else 1e-10
    for b in range(B):
        ref = oadj.grad_noise_alg2(g[b].double().cpu().numpy(), lengths, None, 0, 0, h=h)
        assert relerr(gz[b].double().cpu().numpy(), ref) <= tol
        L = float((w[b] * phi[b].double().cpu() ** 2).sum())
        assert float(gt[b, 0]) * sigma == pytest.approx(2 * L, rel=tol * 10)
        assert float(gt[b, 1]) == 0.0 and float(gt[b, 2]) == 0.0


def test_statistical_covariance_figure3_method(grf):
    """Figure 3's test (covariance of the field at one grid point with all
    others, estimated from samples) for the anisotropic case (d): the estimate
    matches the exact covariance of the sampled law within its Monte Carlo
    error, and shows the anisotropy."""
    dims, lengths, mkln = (64, 64), (4.0, 4.0), (5.0, 3, 1, 1)
    plan = paper_plan(grf, dims, lengths, mkln)
    n = 40000
    est = plan.covariance(seed=0, nsamples=n).cpu().numpy()
    S = spectra.density_on_grid(dims, lengths, spectra.paper_density(*mkln), half=False)
    cn = ogrf.discrete_covariance(dims, lengths, None, 0, 0, h_full=spectra.filter_from_density(dims, lengths, S))
    se = np.sqrt((cn[0, 0] ** 2 + cn ** 2) / n)
    assert np.all(np.abs(est - cn) <= 6 * se), np.max(np.abs(est - cn) / se)
