"""Host-side checks of the torch wrapper, on the CPU: tensors handed to the
library as raw pointers are validated (shape, dtype, device, layout) before
any call, and the autograd Function takes its field count and gradient
placement from its arguments.  A stub plan stands in for the library, so
nothing here touches a GPU."""
import os

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1105_2737_amd", "libgrf.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgrf.so not built")


def _api():
    from paper_1105_2737_amd import api
    return api


def _bare_plan(dims=(8, 6), dtype=torch.float32, device="cpu"):
    """A Plan object without a library handle: only its host-side helpers run."""
    api = _api()
    p = api.Plan.__new__(api.Plan)
    p.dims, p.dtype, p.device, p.handle = tuple(dims), dtype, torch.device(device), None
    return p


def test_out_is_checked():
    p = _bare_plan()
    good = torch.empty((3, 8, 6), dtype=torch.float32)
    assert p._out(good, 3) is good
    with pytest.raises(ValueError, match="shape"):
        p._out(torch.empty((3, 8, 5)), 3)                      # wrong grid: the kernels would write past it
    with pytest.raises(ValueError, match="shape"):
        p._out(torch.empty((2, 8, 6)), 3)                      # too few fields
    big = torch.empty((5, 8, 6))
    assert p._out(big, 3) is big                               # the first 3 fields are written
    with pytest.raises(ValueError, match="float32"):
        p._out(torch.empty((3, 8, 6), dtype=torch.float64), 3)  # would be half written
    with pytest.raises(ValueError, match="contiguous"):
        p._out(torch.empty((3, 6, 8)).transpose(1, 2), 3)
    with pytest.raises(ValueError, match="on"):
        p._out(torch.empty((3, 8, 6), device="meta"), 3)
    with pytest.raises(TypeError):
        p._out([0.0] * 144, 3)


def test_field_inputs_are_checked_and_converted():
    p = _bare_plan(dtype=torch.float64)
    t, b = p._fields("noise", torch.zeros((4, 8, 6), dtype=torch.float32))
    assert b == 4 and t.dtype == torch.float64 and t.is_contiguous()
    t, b = p._fields("noise", torch.zeros((2, 6, 8)).transpose(1, 2))
    assert b == 2 and t.is_contiguous()
    with pytest.raises(ValueError, match="batch, 8, 6"):
        p._fields("noise", torch.zeros((4, 8, 7)))            # wrong grid size: the kernels would read past it
    with pytest.raises(ValueError, match="batch, 8, 6"):
        p._fields("grad_out", torch.zeros((8, 6)))             # missing batch axis


def test_theta_shapes():
    p = _bare_plan()
    assert p._theta(None, 4) is None
    assert p._theta(torch.tensor([1.0, 0.1, 1.5]), 4).shape == (4, 3)
    with pytest.raises(ValueError):
        p._theta(torch.ones(5, 3), 4)


class _StubPlan:
    """Records what the autograd Function asks of the library."""

    def __init__(self, dims=(4, 4)):
        self.dims, self.device, self.dtype = dims, torch.device("cpu"), torch.float32
        self.calls = []

    def sample(self, seed=0, batch=1, theta=None, out=None):
        self.calls.append(("sample", batch, tuple(theta.shape)))
        return theta[:, :1, None].float().expand(batch, *self.dims).clone()

    def sample_from_noise(self, noise, theta=None, out=None):
        self.calls.append(("noise", noise.shape[0], tuple(theta.shape)))
        return noise * theta[:, :1, None].float()

    def backward(self, g, seed=0, theta=None, noise=None, need_noise_grad=False):
        b = g.shape[0]
        self.calls.append(("backward", b, need_noise_grad))
        gt = torch.arange(3 * b, dtype=torch.float64).reshape(b, 3)
        return gt, (torch.ones_like(g) if need_noise_grad else None)


def test_shared_theta_needs_batch():
    api = _api()
    plan = _StubPlan()
    theta = torch.tensor([1.0, 0.1, 1.5], dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="batch"):
        api.GRFSample.apply(theta, plan, 0)                    # a [3] theta is not 3 fields
    phi = api.GRFSample.apply(theta, plan, 0, None, 5)
    assert phi.shape == (5, 4, 4)
    assert plan.calls[-1] == ("sample", 5, (5, 3))
    phi.sum().backward()
    # per-field gradients summed over the fields that share theta
    assert torch.equal(theta.grad, torch.arange(15, dtype=torch.float64).reshape(5, 3).sum(0))


def test_batch_must_match_theta_rows():
    api = _api()
    theta = torch.ones(4, 3, dtype=torch.float64)
    with pytest.raises(ValueError):
        api.GRFSample.apply(theta, _StubPlan(), 0, None, 3)
    with pytest.raises(ValueError):
        api.GRFSample.apply(torch.ones(4, 2, dtype=torch.float64), _StubPlan(), 0)


def test_gradient_lands_on_theta_device_and_dtype():
    api = _api()
    plan = _StubPlan()
    theta = torch.ones(3, 3, dtype=torch.float32, requires_grad=True)   # float32 theta on the CPU
    phi = api.GRFSample.apply(theta, plan, 0)
    phi.sum().backward()
    assert theta.grad.dtype == torch.float32 and theta.grad.device == theta.device
    assert plan.calls[0] == ("sample", 3, (3, 3))


def test_noise_gradient_path():
    api = _api()
    plan = _StubPlan()
    theta = torch.ones(3, dtype=torch.float64, requires_grad=True)
    z = torch.randn(2, 4, 4, requires_grad=True)
    phi = api.GRFSample.apply(theta, plan, 0, z)               # field count from the noise
    assert plan.calls[0] == ("noise", 2, (2, 3))
    phi.sum().backward()
    assert plan.calls[-1] == ("backward", 2, True)
    assert z.grad.shape == z.shape and z.grad.dtype == z.dtype
    assert theta.grad.shape == (3,)
