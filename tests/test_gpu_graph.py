"""Capture of the sampler and the adjoint into a HIP graph (torch.cuda.graph
on the plan's calls): the library allocates nothing, clears nothing with a
memset and never synchronises inside a call, so a captured call replays.
Every replay, with unrelated eager work and synchronisations between the
replays, must give the eager result bit for bit."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                   # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


CASES = [
    dict(dims=(512, 512), batch=300, kw=dict(cov="matern")),                      # two chunks
    dict(dims=(64, 48, 32), batch=5, kw=dict(cov="exponential", length_scale=0.05)),
    dict(dims=(4096,), batch=64, kw=dict(cov="gaussian", length_scale=0.02)),
    dict(dims=(96, 128), batch=7, kw=dict(cov="matern", boundary="dirichlet")),
    dict(dims=(16, 24, 32), batch=3, kw=dict(cov="matern", boundary="neumann")),
    dict(dims=(128, 256), batch=9, kw=dict(cov="matern", draw_order="recursive")),
    dict(dims=(256, 256), batch=6, kw=dict(cov="paper", m=5.0, k=3, l=1, n=1, lengths=(4.0, 4.0))),
    dict(dims=(16, 24, 32), batch=4, kw=dict(cov="matern", alg=1)),             # two-FFT, seven passes
    dict(dims=(360,), batch=8, kw=dict(cov="gaussian", length_scale=0.05, alg=1)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['dims']}-{sorted(c['kw'].items())}")
def test_sample_replays(grf, case):
    kw = dict(case["kw"])
    lengths = kw.pop("lengths", None)
    plan = grf.Plan(case["dims"], lengths=lengths, **kw)
    B = case["batch"]
    ref = plan.sample(seed=17, batch=B).clone()
    out = torch.empty_like(ref)
    g = _capture(lambda: plan.sample(seed=17, batch=B, out=out))
    scratch = torch.empty(1 << 20, device="cuda")
    for k in range(4):
        out.fill_(float("nan"))
        scratch.normal_()                          # unrelated eager work between replays
        _ = plan.sample(seed=3, batch=2)           # and eager calls of the same plan
        _ = scratch.sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k


def test_backward_replays(grf):
    dims, B = (128, 192), 5
    plan = grf.Plan(dims, cov="matern", sigma=1.2, length_scale=0.1, nu=1.5)
    phi = plan.sample(seed=2, batch=B)
    gin = (2 * phi).contiguous()
    gt_ref, gz_ref = plan.backward(gin, seed=2, need_noise_grad=True)
    gt_ref, gz_ref = gt_ref.clone(), gz_ref.clone()
    res = {}

    def step():
        res["gt"], res["gz"] = plan.backward(gin, seed=2, need_noise_grad=True)
    g = _capture(step)
    for k in range(4):
        res["gt"].fill_(float("nan"))
        res["gz"].fill_(float("nan"))
        _ = plan.sample(seed=5, batch=1).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res["gt"], gt_ref), k
        assert torch.equal(res["gz"], gz_ref), k
