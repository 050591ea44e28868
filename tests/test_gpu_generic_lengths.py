"""Grid lengths without a compile-time kernel (any even 2/3/5-smooth N up to
4096 on a leading axis and 16384 on the last axis, Section 3's Input list asks
only for even N_i): the runtime-radix passes against the float64 oracle, for
both algorithms, d = 1, 2, 3, float32 and float64, as the leading axis, the
middle axis and the last axis; large fields; chunked batches give the same
bits; the features that take the listed lengths only refuse the others."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import adjoint as oadj  # noqa: E402
from oracle import grf as ogrf  # noqa: E402
from oracle import noise as onoise  # noqa: E402
from oracle import spectra  # noqa: E402

# leading-axis lengths and last-axis half-lengths that are not in the compiled lists
GEN_COL = [6, 10, 18, 20, 40, 80, 90, 150, 240, 640, 720, 810, 1200, 1280, 1536, 2048, 2700, 4096]
GEN_HALF = [3, 5, 10, 18, 40, 75, 125, 240, 720, 768, 1500, 4096, 6000, 8192]
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


def check(grf, dims, dtype, alg, seed=1, batch=1):
    lengths = tuple(1.0 + 0.25 * i for i in range(len(dims)))
    print(f"generic length: dims {dims} alg {alg} {dtype} batch {batch}", flush=True)
    plan = grf.Plan(dims, lengths=lengths, alg=alg, dtype=dtype, cov="matern", sigma=PARAMS[0],
                    length_scale=PARAMS[1], nu=PARAMS[2])
    out = plan.sample(seed=seed, batch=batch)
    for b in sorted({0, batch - 1}):
        got = out[b].double().cpu().numpy()
        ref = ogrf.sample(dims, lengths, spectra.MATERN, *PARAMS, seed=seed + b, batch=1, alg=alg)[0]
        e = relerr(got, ref)
        assert e <= TOL[dtype], (dims, alg, dtype, b, e)
    return plan, out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("L", GEN_COL)
def test_generic_leading_axis(grf, dtype, L):
    for alg in (2, 1):
        check(grf, (L, 16), dtype, alg)           # axis 1 of d = 2
        check(grf, (4, L, 8), dtype, alg)         # the middle axis of d = 3
        check(grf, (L, 6, 8), dtype, alg)         # axis 1 of d = 3


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("M", GEN_HALF)
def test_generic_last_axis(grf, dtype, M):
    for alg in (2, 1):
        check(grf, (2 * M,), dtype, alg, batch=3)  # d = 1
        check(grf, (8, 2 * M), dtype, alg)
        if M <= 1500:
            check(grf, (4, 6, 2 * M), dtype, alg)


@pytest.mark.parametrize("dims", [(90, 250), (720, 80), (40, 30, 18), (4096, 4096), (2048, 6000)])
def test_generic_mixed_and_large(grf, dims):
    """Every axis off the lists, and large fields (16.8M and 12.3M points)."""
    dtype = torch.float32
    check(grf, dims, dtype, 2, seed=7, batch=1)
    if np.prod(dims) <= 1 << 22:
        check(grf, dims, dtype, 1, seed=7, batch=1)


def test_generic_chunks_same_bits(grf):
    """Cache-sized chunks with a ragged tail give the same bits as one chunk."""
    dims = (720, 90)
    for alg in (2, 1):
        plan = grf.Plan(dims, alg=alg, dtype=torch.float32)
        ref = plan.sample(seed=11, batch=7)
        old = os.environ.get("GRF_CHUNK_BYTES")
        os.environ["GRF_CHUNK_BYTES"] = str(3 * dims[0] * dims[1] * 4)
        try:
            got = plan.sample(seed=11, batch=7)
        finally:
            if old is None:
                del os.environ["GRF_CHUNK_BYTES"]
            else:
                os.environ["GRF_CHUNK_BYTES"] = old
        assert torch.equal(got, ref)
        # field b of a batch is field seed + b on its own
        assert torch.equal(plan.sample(seed=16, batch=1)[0], ref[5])


def test_generic_theta_and_noise_routes(grf):
    """Per-field parameters and a given noise array on a runtime-radix plan."""
    dims = (80, 150)
    plan = grf.Plan(dims, alg=2, dtype=torch.float64)
    theta = torch.tensor([[1.0, 0.15, 1.5], [2.0, 0.1, 0.5]], dtype=torch.float64, device="cuda")
    out = plan.sample(seed=3, batch=2, theta=theta)
    for b in range(2):
        s, ell, nu = theta[b].tolist()
        ref = ogrf.sample(dims, (1.0, 1.0), spectra.MATERN, s, ell, nu, seed=3 + b, batch=1, alg=2)[0]
        assert relerr(out[b].cpu().numpy(), ref) <= 1e-12
    z = plan.noise(seed=3, batch=2)
    assert torch.equal(plan.sample_from_noise(z, theta=theta), out)


def test_generic_refusals(grf):
    from paper_1105_2737_amd import _lib as L
    for kw in (dict(boundary="neumann"), dict(draw_order="recursive")):
        with pytest.raises(L.GRFError) as ei:
            grf.Plan((80, 16), alg=2, dtype=torch.float32, **kw)
        assert ei.value.status == L.GRF_EUNSUPPORTED
    with pytest.raises(L.GRFError) as ei:
        grf.Plan((8192, 16), alg=2, dtype=torch.float32)          # above the leading-axis limit
    assert ei.value.status == L.GRF_EUNSUPPORTED
    with pytest.raises(L.GRFError) as ei:
        grf.Plan((16, 2 * 3 * 7), alg=2, dtype=torch.float32)     # not 2/3/5-smooth
    assert ei.value.status == L.GRF_EINVAL


# (dims, lengths): every axis off the lists, one axis off, a self-mirrored
# column length of 6, odd half-lengths, d = 1 and 3
ADJ_DIMS = [((80, 150), (1.0, 1.5)), ((6, 10), (1.0, 1.0)), ((720, 16), (2.0, 1.0)), ((16, 250), (1.0, 2.0)),
            ((10, 18, 6), (1.0, 1.25, 1.5)), ((4, 40, 16), (1.0, 1.0, 1.0)), ((150,), (1.0,)), ((2 * 1500,), (2.0,))]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("alg", [2, 1])
@pytest.mark.parametrize("dims,lengths", ADJ_DIMS, ids=str)
def test_generic_adjoint(grf, dtype, alg, dims, lengths):
    """dL/dtheta and dL/dz of runtime-radix plans against the float64 oracle,
    each theta component against its own scale, for two fields with generated
    noise, and the same gradients with the noise passed in."""
    params = (1.2, 0.15, 1.5)
    print(f"generic adjoint: dims {dims} alg {alg} {dtype}", flush=True)
    plan = grf.Plan(dims, lengths=lengths, alg=alg, dtype=dtype, cov="matern", sigma=params[0],
                    length_scale=params[1], nu=params[2])
    B, seed = 2, 5
    g = torch.randn((B,) + dims, dtype=torch.float64, generator=torch.Generator().manual_seed(9))
    gt, gz = plan.backward(g, seed=seed, need_noise_grad=True)
    gt = gt.cpu().numpy()
    gz = gz.double().cpu().numpy()
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    tag = onoise.TAG_ALG2 if alg == 2 else onoise.TAG_ALG1
    for b in range(B):
        z = onoise.field_noise(dims, seed + b, tag)
        gb = g[b].numpy()
        if alg == 2:
            rt = oadj.grad_theta_alg2(z, gb, lengths, spectra.MATERN, *params)
            rz = oadj.grad_noise_alg2(gb, lengths, spectra.MATERN, *params)
        else:
            rt = oadj.grad_theta_alg1(z, gb, lengths, spectra.MATERN, *params)
            rz = oadj.grad_noise_alg1(gb, lengths, spectra.MATERN, *params)
        # each component against its own scale: the sum of its absolute terms
        # w (h/2) |dlogS/dtheta| |Re(xi conj G)|, which bounds the rounding error
        P = int(np.prod(dims))
        xi = ogrf.hermitian_noise(z) if alg == 2 else np.fft.rfftn(z) / np.sqrt(P)
        core = oadj.half_weights(dims) * np.abs(np.real(xi * np.conj(np.fft.rfftn(gb))))
        h = spectra.filter_h(dims, lengths, spectra.MATERN, *params, half=True)
        dlog = spectra.dlog_spectral_density(spectra.MATERN, spectra.freq2_grid(dims, lengths, half=True),
                                             len(dims), *params)
        for c in range(3):
            scale = float(np.sum(0.5 * h * np.abs(dlog[c]) * core))
            assert abs(gt[b, c] - rt[c]) <= tol * scale, (b, c, gt[b], rt, scale)
        assert relerr(gz[b], rz) <= tol, (b, relerr(gz[b], rz))
    z = plan.noise(seed=seed, batch=B)
    gt2, gz2 = plan.backward(g, noise=z, need_noise_grad=True)
    assert np.allclose(gt2.cpu().numpy(), gt, rtol=tol, atol=0)
    assert relerr(gz2.double().cpu().numpy(), gz) <= tol


def test_generic_adjoint_sigma_identity(grf):
    """sigma dL/dsigma = 2 L for L = sum w phi^2 (phi is linear in sigma), on a
    larger runtime-radix grid with per-field parameters."""
    dims = (720, 240)
    plan = grf.Plan(dims, dtype=torch.float64, cov="matern")
    th = torch.tensor([[1.0, 0.1, 1.5], [0.5, 0.2, 0.7]], dtype=torch.float64)
    phi = plan.sample(seed=2, batch=2, theta=th)
    w = torch.rand(phi.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(1)).to(phi.device)
    gt, _ = plan.backward(2 * w * phi, seed=2, theta=th)
    L = (w * phi ** 2).sum(dim=(1, 2))
    np.testing.assert_allclose((gt[:, 0].cpu() * th[:, 0]).numpy(), 2 * L.cpu().numpy(), rtol=1e-10)


@pytest.mark.parametrize("alg", [2, 1])
@pytest.mark.parametrize("dims", [(80, 150), (10, 18, 6)], ids=str)
def test_generic_adjoint_chunks_same_bits(grf, alg, dims):
    """The adjoint over cache-sized chunks (2 fields each, a ragged tail)
    gives the same bits as over one chunk, noise gradient included."""
    plan = grf.Plan(dims, alg=alg, dtype=torch.float32, cov="matern")
    g = torch.randn((5,) + dims, generator=torch.Generator().manual_seed(3)).cuda()
    ref_t, ref_z = plan.backward(g, seed=4, need_noise_grad=True)
    old = os.environ.get("GRF_CHUNK_BYTES")
    os.environ["GRF_CHUNK_BYTES"] = str(2 * int(np.prod(dims)) * 4 + 8)
    try:
        t2, z2 = plan.backward(g, seed=4, need_noise_grad=True)
    finally:
        if old is None:
            del os.environ["GRF_CHUNK_BYTES"]
        else:
            os.environ["GRF_CHUNK_BYTES"] = old
    assert torch.equal(ref_t, t2) and torch.equal(ref_z, z2)
