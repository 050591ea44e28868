"""The allocation-free sampler entry point against grf_sample with a caller
workspace, through the C ABI: same plan, seed and per-field parameters give
the same bits, on two calls in a row (the second with fewer fields, so that
stale records of the first call would show), for d = 2 and d = 3 and both
precisions; the field-count limit is enforced before any launch."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _theta(batch, seed):
    rng = np.random.default_rng(seed)
    th = np.stack([rng.uniform(0.5, 2.0, batch), rng.uniform(0.05, 0.2, batch), rng.choice([0.5, 1.5, 2.5], batch)], 1)
    return torch.tensor(th, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("dims,dtype", [((96, 128), torch.float32), ((64, 48, 48), torch.float32),
                                        ((96, 128), torch.float64), ((512, 512), torch.float32)])
def test_noalloc_matches_sample(dims, dtype):
    import paper_1105_2737_amd as grf
    from paper_1105_2737_amd import _lib as L
    plan = grf.Plan(dims, alg=2, dtype=dtype, cov="matern")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for batch, seed in ((37, 11), (5, 3)):
        print(f"noalloc {dims} {dtype} batch {batch} seed {seed}", flush=True)
        theta = _theta(batch, seed)
        ref = plan.sample(seed=seed, batch=batch, theta=theta)
        got = torch.full_like(ref, float("nan"))
        L.grf_sample_noalloc(plan.handle, seed, batch, _ptr(theta), _ptr(got), stream)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"batch {batch}: max diff {(got - ref).abs().max().item()}"
    # no per-field parameters: the plan's own (no scratch used)
    ref = plan.sample(seed=2, batch=3)
    got = torch.empty_like(ref)
    L.grf_sample_noalloc(plan.handle, 2, 3, None, _ptr(got), stream)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_two_fft_and_limits():
    import paper_1105_2737_amd as grf
    from paper_1105_2737_amd import _lib as L
    plan = grf.Plan((64, 64), alg=1, dtype=torch.float32, cov="matern")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    theta = _theta(9, 1)
    ref = plan.sample(seed=4, batch=9, theta=theta)
    got = torch.empty_like(ref)
    L.grf_sample_noalloc(plan.handle, 4, 9, _ptr(theta), _ptr(got), stream)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    # over the limit with per-field parameters: rejected on the host, nothing written
    big = L.GRF_NOALLOC_MAX_FIELDS + 1
    out = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(L.GRFError) as ei:
        L.grf_sample_noalloc(plan.handle, 0, big, _ptr(theta), _ptr(out), stream)
    assert ei.value.status == L.GRF_EINVAL
    assert "GRF_NOALLOC_MAX_FIELDS" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    # empty batch: a no-op
    L.grf_sample_noalloc(plan.handle, 0, 0, _ptr(theta), _ptr(out), stream)
