"""GPU parity: the HIP library against the float64 oracle on the same seeded
noise.  Error metric per field (the one the float32 target is stated in):
max_j |phi_gpu - phi_oracle| / max_j |phi_oracle|; float32 <= 1e-5,
float64 <= 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import grf as ogrf  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
KIND = {"gaussian": spectra.GAUSSIAN, "matern": spectra.MATERN, "exponential": spectra.EXPONENTIAL}


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def oracle_fields(dims, lengths, cov, params, seed, batch, alg, idx=None):
    idx = range(batch) if idx is None else idx
    return {b: ogrf.sample(dims, lengths, KIND[cov], *params, seed=seed + b, batch=1, alg=alg)[0] for b in idx}


def test_philox_bit_exact(grf):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]]
    dc = torch.from_numpy(ctr.view(np.int32)).cuda().contiguous()
    out = torch.empty_like(dc)
    for seed in [0, 1, 0xA4093822 | (0x299F31D0 << 32), 2 ** 64 - 1]:
        grf.grf_debug_philox(seed, dc.data_ptr(), 4096, out.data_ptr(), None)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        want = onoise.philox_raw(seed, ctr.astype(np.uint64))
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("alg", [1, 2])
def test_noise_matches_contract(grf, dtype, alg):
    dims = (24, 48)
    plan = grf.Plan(dims, alg=alg, dtype=dtype)
    z = plan.noise(seed=5, batch=3).double().cpu().numpy()
    ref = onoise.batch_noise(dims, 5, 3, 1 if alg == 2 else 0)
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert np.abs(z - ref).max() <= tol * np.abs(ref).max()


def test_noise_box_muller_tail(grf):
    """Float32 normals stay within 4e-6 absolute of the float64 contract,
    including the draws with u -> 1 where -2 ln u is taken from a series
    (1 - u < 2^-13, i.e. radius r < 2^-6) and the band just above it where
    the rounding of u to float32 costs up to 2^-25 / r.  Adjacent pairs along
    the last axis are one Box-Muller pair; 4M normals hold ~256 pairs in the
    series range."""
    dims = (1024, 1024)
    plan = grf.Plan(dims, alg=2, dtype=torch.float32)
    z = plan.noise(seed=77, batch=4).double().cpu().numpy()
    ref = onoise.batch_noise(dims, 77, 4, 1)
    err = np.abs(z - ref)
    assert err.max() <= 4e-6
    r = np.hypot(ref[..., 0::2], ref[..., 1::2])
    tail = r < 2.0 ** -6
    assert tail.sum() >= 150
    pair_err = np.maximum(err[..., 0::2], err[..., 1::2])
    assert pair_err[tail].max() <= 1e-6
    band = (r >= 2.0 ** -6) & (r < 2.0 ** -3)
    assert band.sum() >= 5000 and pair_err[band].max() <= 4e-6


CASES_2D = [
    ((64, 64), (1.0, 1.0), "matern", (1.0, 0.1, 1.5)),
    ((96, 128), (1.0, 2.0), "gaussian", (1.3, 0.07, 0.5)),
    ((360, 64), (1.0, 1.0), "exponential", (0.8, 0.05, 0.5)),
    ((128, 1000), (2.0, 1.0), "matern", (1.0, 0.05, 2.5)),
    ((1000, 48), (1.0, 1.0), "matern", (1.0, 0.2, 0.5)),
    ((8, 24), (1.0, 1.0), "matern", (1.0, 0.3, 1.5)),
    ((12, 8), (1.0, 1.0), "gaussian", (1.0, 0.2, 1.5)),
    ((4, 720), (1.0, 1.0), "matern", (1.0, 0.1, 1.5)),
]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("alg", [2, 1])
@pytest.mark.parametrize("case", CASES_2D, ids=lambda c: "x".join(map(str, c[0])) + "-" + c[2])
def test_2d_against_oracle(grf, dtype, alg, case):
    dims, lengths, cov, params = case
    batch, seed = 3, 11
    print(f"case {dims} alg{alg} {dtype} {cov}", flush=True)
    plan = grf.Plan(dims, lengths=lengths, alg=alg, dtype=dtype, cov=cov, sigma=params[0],
                    length_scale=params[1], nu=params[2])
    got = plan.sample(seed=seed, batch=batch).double().cpu().numpy()
    ref = oracle_fields(dims, lengths, cov, params, seed, batch, alg)
    for b in range(batch):
        e = relerr(got[b], ref[b])
        print(f"  field {b}: rel err {e:.3e}", flush=True)
        assert e <= TOL[dtype]


CASES_3D = [
    ((16, 24, 32), (1.0, 1.0, 1.0), "exponential", (1.0, 0.05, 0.5)),
    ((64, 48, 96), (1.0, 2.0, 1.0), "matern", (1.0, 0.1, 1.5)),
    ((12, 256, 8), (1.0, 1.0, 1.0), "gaussian", (1.0, 0.1, 0.5)),
]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("case", CASES_3D, ids=lambda c: "x".join(map(str, c[0])))
def test_3d_against_oracle(grf, dtype, case):
    dims, lengths, cov, params = case
    print(f"case {dims} {dtype}", flush=True)
    plan = grf.Plan(dims, lengths=lengths, alg=2, dtype=dtype, cov=cov, sigma=params[0], length_scale=params[1],
                    nu=params[2])
    got = plan.sample(seed=3, batch=2).double().cpu().numpy()
    ref = oracle_fields(dims, lengths, cov, params, 3, 2, 2)
    for b in range(2):
        assert relerr(got[b], ref[b]) <= TOL[dtype]


def test_config1_fp64_exact(grf):
    """64 x 64, two-FFT algorithm in float64, Gaussian l = 0.05, seed 0."""
    plan = grf.Plan((64, 64), alg=1, dtype=torch.float64, cov="gaussian", sigma=1.0, length_scale=0.05)
    got = plan.sample(seed=0, batch=1).cpu().numpy()[0]
    ref = ogrf.sample((64, 64), (1, 1), spectra.GAUSSIAN, 1.0, 0.05, seed=0, batch=1, alg=1)[0]
    assert relerr(got, ref) <= 1e-12


@pytest.mark.parametrize("alg", [1, 2])
def test_from_noise_equals_generated(grf, alg):
    dims = (96, 64)
    for dtype in (torch.float32, torch.float64):
        plan = grf.Plan(dims, alg=alg, dtype=dtype)
        z = plan.noise(seed=9, batch=4)
        a = plan.sample(seed=9, batch=4)
        b = plan.sample_from_noise(z)
        torch.testing.assert_close(a, b, rtol=0, atol=0)


@pytest.mark.parametrize("alg", [1, 2])
def test_batch_invariance_and_determinism(grf, alg):
    dims = (128, 96)
    plan = grf.Plan(dims, alg=alg)
    full = plan.sample(seed=100, batch=7)
    again = plan.sample(seed=100, batch=7)
    assert torch.equal(full, again)
    for b in (0, 3, 6):
        one = plan.sample(seed=100 + b, batch=1)
        assert torch.equal(full[b], one[0])


def test_per_field_theta(grf):
    dims = (64, 96)
    plan = grf.Plan(dims, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5)
    theta = torch.tensor([[1.0, 0.1, 1.5], [2.0, 0.05, 0.5], [0.5, 0.2, 2.5]], dtype=torch.float64)
    got = plan.sample(seed=1, batch=3, theta=theta.cuda()).double().cpu().numpy()
    for b in range(3):
        ref = ogrf.sample(dims, (1, 1), spectra.MATERN, *theta[b].tolist(), seed=1 + b, batch=1, alg=2)[0]
        assert relerr(got[b], ref) <= 1e-5
    # same parameters through the record path and the plan default: same bits
    d0 = plan.sample(seed=1, batch=1)
    assert torch.equal(d0[0], plan.sample(seed=1, batch=1, theta=theta[:1].cuda())[0])


def test_batch_zero_is_noop(grf):
    plan = grf.Plan((64, 64))
    out = torch.full((1, 64, 64), 7.0, device="cuda")
    plan.sample(seed=0, batch=0, out=out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dims", [(64, 96), (128, 64), (360, 1000)])
def test_backward_against_oracle(grf, dtype, dims):
    cov, params = "matern", (1.0, 0.1, 1.5)
    batch, seed = 2, 4
    plan = grf.Plan(dims, alg=2, dtype=dtype, cov=cov, sigma=params[0], length_scale=params[1], nu=params[2])
    rng = np.random.default_rng(1)
    w = rng.uniform(0, 1, size=(batch,) + dims)
    phi = plan.sample(seed=seed, batch=batch).double().cpu().numpy()
    g = 2 * w * phi
    gt, gz = plan.backward(torch.from_numpy(g), seed=seed, need_noise_grad=False)
    gt = gt.cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-10
    for b in range(batch):
        z = onoise.field_noise(dims, seed + b, onoise.TAG_ALG2)
        ref = oadj.grad_theta_alg2(z, g[b], (1, 1), spectra.MATERN, *params)
        for i in range(3):
            assert abs(gt[b, i] - ref[i]) <= tol * np.abs(ref).max(), (b, i, gt[b], ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noise_gradient_against_oracle(grf, dtype):
    dims, params = (64, 48), (1.2, 0.1, 2.5)
    plan = grf.Plan(dims, alg=2, dtype=dtype, cov="matern", sigma=params[0], length_scale=params[1], nu=params[2])
    z = plan.noise(seed=2, batch=2)
    g = torch.randn((2,) + dims, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    gt, gz = plan.backward(g, noise=z, need_noise_grad=True)
    gz = gz.double().cpu().numpy()
    tol = 2e-5 if dtype == torch.float32 else 1e-12
    for b in range(2):
        ref = oadj.grad_noise_alg2(g[b].numpy(), (1, 1), spectra.MATERN, *params)
        assert np.abs(gz[b] - ref).max() <= tol * np.abs(ref).max()


def test_autograd_function(grf):
    dims = (64, 64)
    plan = grf.Plan(dims, alg=2, dtype=torch.float32, cov="matern")
    theta = torch.tensor([[1.0, 0.1, 1.5]] * 2, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.rand((2,) + dims, device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    phi = grf.GRFSample.apply(theta, plan, 3)
    loss = (w * phi.double() ** 2).sum()
    loss.backward()
    # sigma dL/dsigma = 2 L per field (phi is linear in sigma)
    Lb = (w * phi.double() ** 2).sum(dim=(1, 2))
    np.testing.assert_allclose(theta.grad[:, 0].cpu().numpy(), (2 * Lb / theta[:, 0]).detach().cpu().numpy(),
                               rtol=1e-5)


@pytest.mark.parametrize("dims", [(512, 512), (96, 96)])
def test_chunk_schedule_ragged_tail(grf, dims):
    """Cache-sized chunks with a ragged last chunk (3+3+3 and 4+4+1 fields)
    give the same bits as one chunk; the launch count follows the chunking."""
    import os
    plan = grf.Plan(dims, alg=2)
    old = dict(os.environ)
    try:
        ref = plan.sample(seed=5, batch=9)
        assert grf.grf_sample_stage_count(plan.handle, 9) == 2
        os.environ["GRF_CHUNK_BYTES"] = str(3 * dims[0] * dims[1] * 4)   # 3 fields per chunk
        got = plan.sample(seed=5, batch=9)
        assert grf.grf_sample_stage_count(plan.handle, 9) == 6
        os.environ["GRF_CHUNK_BYTES"] = str(4 * dims[0] * dims[1] * 4)   # 4, 4, 1
        got2 = plan.sample(seed=5, batch=9)
    finally:
        os.environ.clear()
        os.environ.update(old)
    assert torch.equal(got, ref)
    assert torch.equal(got2, ref)


def _with_env(env, fn):
    import os
    old = dict(os.environ)
    try:
        os.environ.update(env)
        return fn()
    finally:
        os.environ.clear()
        os.environ.update(old)


CHUNK_CASES = [((512, 512), 2, torch.float32), ((96, 128), 1, torch.float32), ((32, 48, 64), 2, torch.float32),
               ((64, 96), 2, torch.float64), ((64, 96), 1, torch.float64)]


@pytest.mark.parametrize("dims,alg,dtype", CHUNK_CASES, ids=lambda c: str(c))
def test_chunked_schedule_matches_unchunked(grf, dims, alg, dtype):
    """Cache-sized chunks (here 3 fields, last chunk ragged) give the same bits as
    one launch per pass, with shared and per-field theta and with supplied noise."""
    P = int(np.prod(dims))
    esz = 4 if dtype == torch.float32 else 8
    B = 7
    cov = "exponential" if len(dims) == 3 else "matern"
    plan = grf.Plan(dims, alg=alg, dtype=dtype, cov=cov)
    g = torch.Generator().manual_seed(3)
    theta = torch.stack([1 + torch.rand(B, generator=g), 0.05 + 0.1 * torch.rand(B, generator=g),
                         0.5 + 2 * torch.rand(B, generator=g)], 1).double()
    z = plan.noise(seed=40, batch=B)
    big = {"GRF_CHUNK_BYTES": str(1 << 40)}
    small = {"GRF_CHUNK_BYTES": str(3 * P * esz)}
    for run in (lambda: plan.sample(seed=11, batch=B), lambda: plan.sample(seed=11, batch=B, theta=theta),
                lambda: plan.sample_from_noise(z)):
        ref = _with_env(big, run)
        got = _with_env(small, run)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    nper = 2 if (alg == 2 and len(dims) == 2) else 3
    n = _with_env(small, lambda: grf.grf_sample_stage_count(plan.handle, B))
    assert n == 3 * nper
    info = _with_env(small, lambda: [grf.grf_sample_stage_info(plan.handle, B, s) for s in range(n)])
    assert [(f, c) for _, f, c in info[::nper]] == [(0, 3), (3, 3), (6, 1)]
    # one-FFT 512^2 float32: the last-axis pass also runs the column transform's last stage
    split = dims == (512, 512) and alg == 2 and dtype == torch.float32
    assert info[nper - 1][0] == (112 if split else grf.GRF_PASS_ROW_C2R)
    assert _with_env(big, lambda: grf.grf_sample_stage_count(plan.handle, B)) == nper


@pytest.mark.parametrize("order", ["counter", "recursive"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_split_last_stage_matches_unsplit(grf, dtype, order):
    """512 x 512, one-FFT: the column pass without its last radix stage plus the
    last-axis pass that runs it (kinds 111 or 113, then 112) give the bits of
    the column pass plus the plain complex-to-real (GRF_SPLIT=0), with seeds,
    per-field theta and supplied noise, over a ragged chunk schedule."""
    dims, B = (512, 512), 5
    esz = 4 if dtype == torch.float32 else 8
    plan = grf.Plan(dims, alg=2, dtype=dtype, cov="matern", sigma=1.0, length_scale=0.1, nu=1.5, draw_order=order)
    gen, part = ((grf.GRF_PASS_COL_GEN_INV, 111) if order == "counter" else (grf.GRF_PASS_COL_SEQ_INV, 113))
    g = torch.Generator().manual_seed(8)
    theta = torch.stack([1 + torch.rand(B, generator=g), 0.05 + 0.1 * torch.rand(B, generator=g),
                         0.5 + 2 * torch.rand(B, generator=g)], 1).double()
    z = plan.noise(seed=21, batch=B)
    chunk = {"GRF_CHUNK_BYTES": str(2 * dims[0] * dims[1] * esz)}   # 2, 2, 1 fields
    kinds = _with_env(chunk, lambda: [grf.grf_sample_stage_info(plan.handle, B, s)[0]
                                      for s in range(grf.grf_sample_stage_count(plan.handle, B))])
    assert kinds == [part, 112] * 3
    off = _with_env(dict(chunk, GRF_SPLIT="0"), lambda: [grf.grf_sample_stage_info(plan.handle, B, s)[0]
                                                        for s in range(grf.grf_sample_stage_count(plan.handle, B))])
    assert off == [gen, grf.GRF_PASS_ROW_C2R] * 3
    for run in (lambda: plan.sample(seed=13, batch=B), lambda: plan.sample(seed=2, batch=B, theta=theta),
                lambda: plan.sample_from_noise(z)):
        got = _with_env(chunk, run)
        ref = _with_env(dict(chunk, GRF_SPLIT="0"), run)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    if order == "counter":   # and against the oracle, two fields (the recursive order's oracle test is its own)
        ref = oracle_fields(dims, (1.0, 1.0), "matern", (1.0, 0.1, 1.5), 13, 2, 2)
        got = plan.sample(seed=13, batch=2).double().cpu().numpy()
        for b in range(2):
            assert relerr(got[b], ref[b]) <= TOL[dtype]
