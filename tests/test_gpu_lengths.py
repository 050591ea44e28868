"""Every supported transform length against the float64 oracle: the column
lengths (generation pass along axis 1, the middle-axis pass of d = 3, the
adjoint's column kernel, the two-FFT algorithm's column passes) and the row
half-lengths (last-axis pass, the 1D kernels, the adjoint's last-axis pass,
the two-FFT algorithm's noise pass), for periodic and reflecting plans, in
float32 and float64."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import grf as ogrf  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import reflect  # noqa: E402
from oracle import spectra  # noqa: E402

COL = [4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 180, 256, 360, 384, 500, 512, 768, 1000, 1024]
ROW_HALF = [2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 180, 192, 256, 360, 384, 500, 512, 1024, 2048]
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
PARAMS = (1.0, 0.15, 1.5)


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def periodic(grf, dims, dtype):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, cov="matern", sigma=PARAMS[0], length_scale=PARAMS[1],
                    nu=PARAMS[2])
    got = plan.sample(seed=1, batch=1)[0].double().cpu().numpy()
    ref = ogrf.sample(dims, lengths, spectra.MATERN, *PARAMS, seed=1, batch=1, alg=2)[0]
    assert relerr(got, ref) <= TOL[dtype], (dims, dtype, relerr(got, ref))
    # adjoint: dL/dtheta for L = sum phi^2 / 2
    g = torch.from_numpy(ref)[None]
    gt, _ = plan.backward(g.to(dtype), seed=1)
    z = onoise.field_noise(dims, 1, onoise.TAG_ALG2)
    rg = oadj.grad_theta_alg2(z, g[0].to(dtype).double().numpy(), lengths, spectra.MATERN, *PARAMS)
    assert np.abs(gt[0].cpu().numpy() - rg).max() <= 10 * TOL[dtype] * np.abs(rg).max(), (dims, dtype)


def two_fft(grf, dims, dtype):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    plan = grf.Plan(dims, lengths=lengths, alg=1, dtype=dtype, cov="matern", sigma=PARAMS[0],
                    length_scale=PARAMS[1], nu=PARAMS[2])
    got = plan.sample(seed=3, batch=1)[0].double().cpu().numpy()
    ref = ogrf.sample(dims, lengths, spectra.MATERN, *PARAMS, seed=3, batch=1, alg=1)[0]
    assert relerr(got, ref) <= TOL[dtype], (dims, dtype, relerr(got, ref))


def reflecting(grf, dims, dtype):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    sine = tuple(i % 2 == 0 for i in range(len(dims)))
    plan = grf.Plan(dims, lengths=lengths, dtype=dtype, boundary=tuple("dirichlet" if x else "neumann" for x in sine),
                    cov="matern", sigma=PARAMS[0], length_scale=PARAMS[1], nu=PARAMS[2])
    got = plan.sample(seed=2, batch=1)[0].double().cpu().numpy()
    ref = reflect.sample(dims, lengths, sine, seed=2, batch=1, kind=spectra.MATERN, sigma=PARAMS[0], ell=PARAMS[1],
                         nu=PARAMS[2])[0]
    assert relerr(got, ref) <= TOL[dtype], (dims, dtype, relerr(got, ref))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("L", COL)
def test_column_length(grf, dtype, L):
    periodic(grf, (L, 16), dtype)
    periodic(grf, (4, L, 8), dtype)
    two_fft(grf, (L, 16), dtype)
    two_fft(grf, (4, L, 8), dtype)
    reflecting(grf, (L, 16), dtype)
    reflecting(grf, (4, L, 8), dtype)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("M", ROW_HALF)
def test_row_length(grf, dtype, M):
    periodic(grf, (8, 2 * M), dtype)
    periodic(grf, (2 * M,), dtype)
    two_fft(grf, (8, 2 * M), dtype)
    two_fft(grf, (2 * M,), dtype)
    reflecting(grf, (8, 2 * M), dtype)
    reflecting(grf, (2 * M,), dtype)
