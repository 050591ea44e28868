"""torch-facing wrapper of the C ABI: plans, sampling and the autograd Function.

torch provides device memory (the caching allocator) and the current stream;
the library does all the work on that stream."""
import ctypes

import torch

from . import _lib as L

DRAW_ORDERS = {"counter": L.GRF_DRAW_COUNTER, "recursive": L.GRF_DRAW_RECURSIVE}
BOUNDARIES = {"periodic": L.GRF_BC_PERIODIC, "neumann": L.GRF_BC_NEUMANN, "dirichlet": L.GRF_BC_DIRICHLET}
COV_KINDS = {"gaussian": L.GRF_COV_GAUSSIAN, "matern": L.GRF_COV_MATERN, "exponential": L.GRF_COV_EXPONENTIAL,
             "paper": L.GRF_COV_PAPER, "tabulated": L.GRF_COV_TABULATED}
ALGS = {1: L.GRF_ALG_TWO_FFT, 2: L.GRF_ALG_ONE_FFT, "two_fft": L.GRF_ALG_TWO_FFT, "one_fft": L.GRF_ALG_ONE_FFT}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(name, t, shape, dtype, device):
    """A tensor handed to the library as a raw pointer must be exactly what the
    kernels will read or write: shape, dtype, device and a dense layout."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A sampling plan: grid, domain, algorithm, precision and covariance family.

    dims: (N_1, ..., N_d), d in {1, 2, 3}, all even; lengths: edge lengths
    (default the unit torus); alg: 2 = one-FFT (Hermitian), 1 = two-FFT;
    dtype: torch.float32 or torch.float64; cov: 'gaussian' | 'matern' |
    'exponential' with default parameters sigma, length_scale, nu; 'paper'
    (the family of Section 4, eq. (5): S = sigma^2 (m^{kl} + (sum p_i^{2k})^l)^{-n},
    parameters m, k, l, n); 'tabulated' (S at the half-spectrum frequencies,
    `spectrum` of shape dims[:-1] + (N_d/2 + 1,), float64).
    boundary: 'periodic' (default), or per axis 'neumann' / 'dirichlet' (one
    string for all axes or a sequence): the cosine / sine transform variant
    on the cell-centred grid of [0, l_i] (one-transform method only); a
    tabulated S then has the field's shape (the slot grid).
    draw_order: 'counter' (default), or 'recursive': the normals in the draw
    order of the recursive algorithm of Section 3, from one sequence per field
    (plan.noise(seed) in row-major order; one-FFT, periodic).
    """

    def __init__(self, dims, lengths=None, alg=2, dtype=torch.float32, cov="matern", sigma=1.0,
                 length_scale=0.1, nu=1.5, device=None, m=1.0, k=1, l=1, n=1, spectrum=None, boundary="periodic",
                 draw_order="counter"):
        dims = tuple(int(n) for n in dims)
        lengths = tuple(float(v) for v in (lengths or (1.0,) * len(dims)))
        if len(lengths) != len(dims):
            raise ValueError("lengths must match dims")
        self.dims, self.lengths = dims, lengths
        self.alg = ALGS[alg]
        self.dtype = dtype
        self.cov = cov
        self.params = (float(sigma), float(length_scale), float(nu))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        d = L.grf_plan_desc()
        d.ndim = len(dims)
        d.alg = self.alg
        d.dtype = L.GRF_F32 if dtype == torch.float32 else L.GRF_F64
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        d.cov_kind = COV_KINDS[cov]
        for i, (ni, li) in enumerate(zip(dims, lengths)):
            d.dims[i] = ni
            d.lengths[i] = li
        d.sigma, d.length_scale, d.nu = self.params
        d.m, d.k, d.l, d.n = float(m), int(k), int(l), int(n)
        bcs = (boundary,) * len(dims) if isinstance(boundary, str) else tuple(boundary)
        if len(bcs) != len(dims):
            raise ValueError("boundary must be one name or one per axis")
        for i, b in enumerate(bcs):
            d.bc[i] = BOUNDARIES[b]
        self.boundary = bcs
        d.draw_order = DRAW_ORDERS[draw_order]
        self.reflect = any(b != "periodic" for b in bcs)
        spec = None
        if cov == "tabulated":
            import numpy as np
            spec = np.ascontiguousarray(np.asarray(spectrum, dtype=np.float64))
            want = dims if self.reflect else dims[:-1] + (dims[-1] // 2 + 1,)
            if spec.shape != want:
                raise ValueError(f"spectrum must have shape {want}, got {spec.shape}")
            d.spectrum = spec.ctypes.data
        with torch.cuda.device(self.device):
            self.handle = L.grf_plan_create(d)   # the library copies the spectrum

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.lib.grf_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # -- helpers -------------------------------------------------------------
    def _empty(self, batch):
        return torch.empty((batch,) + self.dims, dtype=self.dtype, device=self.device)

    def _out(self, out, batch):
        """The output buffer: [n, *dims] with n >= batch (fields 0 .. batch-1 are
        written), the plan's dtype and device, dense."""
        if out is None:
            return self._empty(batch)
        if isinstance(out, torch.Tensor) and out.dim() == len(self.dims) + 1 and out.shape[0] >= batch:
            return _check("out", out, (out.shape[0],) + self.dims, self.dtype, self.device)
        return _check("out", out, (batch,) + self.dims, self.dtype, self.device)

    def _fields(self, name, t):
        """A [batch, *dims] input (noise, upstream gradient) in the plan's dtype
        on the plan's device, dense; returns it and the batch size."""
        t = torch.as_tensor(t).to(device=self.device, dtype=self.dtype).contiguous()
        if t.dim() != len(self.dims) + 1 or tuple(t.shape[1:]) != self.dims:
            raise ValueError(f"{name} must have shape [batch, {', '.join(map(str, self.dims))}], "
                             f"got {tuple(t.shape)}")
        return t, int(t.shape[0])

    def _workspace(self, batch, op):
        n = L.grf_workspace_size(self.handle, batch, op)
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        return ws, n

    def _theta(self, theta, batch):
        if theta is None:
            return None
        theta = torch.as_tensor(theta, dtype=torch.float64, device=self.device)
        if theta.dim() == 1:
            theta = theta.expand(batch, 3)
        if theta.shape != (batch, 3):
            raise ValueError(f"theta must be [batch, 3] or [3], got {tuple(theta.shape)}")
        return theta.contiguous()

    # -- sampling ------------------------------------------------------------
    def sample(self, seed=0, batch=1, theta=None, out=None):
        """Fields seed .. seed+batch-1, shape [batch, *dims]."""
        batch = int(batch)
        if batch < 0:
            raise ValueError("batch must be >= 0")
        th = self._theta(theta, batch)
        out = self._out(out, batch)
        ws, n = self._workspace(batch, L.GRF_OP_SAMPLE)
        L.grf_sample(self.handle, int(seed) & (2 ** 64 - 1), batch, _ptr(th), _ptr(out), _ptr(ws), n, _stream())
        return out

    def sample_from_noise(self, noise, theta=None, out=None):
        noise, batch = self._fields("noise", noise)
        th = self._theta(theta, batch)
        out = self._out(out, batch)
        if out.data_ptr() == noise.data_ptr() and batch > 0:
            raise ValueError("noise and out must not alias")
        ws, n = self._workspace(batch, L.GRF_OP_SAMPLE)
        L.grf_sample_from_noise(self.handle, _ptr(noise), batch, _ptr(th), _ptr(out), _ptr(ws), n, _stream())
        return out

    def tune(self, batch=1, out=None):
        """Time the candidate kernels of every pass on a chunk of `batch` fields
        (written into `out`, or a scratch buffer) and keep the fastest; the
        choices are appended to the GRF_TUNE_CACHE file when set."""
        batch = int(batch)
        out = self._out(out, batch)
        L.grf_plan_tune(self.handle, batch, _ptr(out), _stream())

    def tune_choice(self, pass_, length):
        return L.grf_plan_tune_choice(self.handle, int(pass_), int(length))

    def covariance(self, seed=0, nsamples=1):
        """Statistical covariance (1/n) sum_b phi_b(x_0) phi_b(x) over fields
        seed .. seed+n-1 (float64 tensor of the field's shape)."""
        cov = torch.empty(self.dims, dtype=torch.float64, device=self.device)
        ws, n = self._workspace(int(nsamples), L.GRF_OP_COVARIANCE)
        L.grf_covariance(self.handle, int(seed) & (2 ** 64 - 1), int(nsamples), _ptr(cov), _ptr(ws), n, _stream())
        return cov

    def noise(self, seed=0, batch=1):
        out = self._empty(batch)
        L.grf_noise(self.handle, int(seed) & (2 ** 64 - 1), batch, _ptr(out), _stream())
        return out

    def spectrum(self, seed=0, batch=1):
        """The half-spectrum A = h xi the one-FFT sampler transforms, complex
        [batch, N_1, ..., N_{d-1}, N_d / 2]; slot 0 holds A(k, 0) + i A(k, N_d/2)."""
        M = self.dims[-1] // 2
        out = torch.empty((batch,) + tuple(self.dims[:-1]) + (M, 2), dtype=self.dtype, device=self.device)
        L.grf_debug_spectrum(self.handle, int(seed) & (2 ** 64 - 1), batch, _ptr(out), _stream())
        return torch.view_as_complex(out)

    def backward(self, grad_out, seed=0, theta=None, noise=None, need_noise_grad=False):
        """(dL/dtheta [batch, 3] float64, dL/dz or None) for either algorithm."""
        grad_out, batch = self._fields("grad_out", grad_out)
        th = self._theta(theta, batch)
        if noise is not None:
            noise, nb = self._fields("noise", noise)
            if nb != batch:
                raise ValueError(f"noise has {nb} fields, grad_out {batch}")
        gt = torch.empty((batch, 3), dtype=torch.float64, device=self.device)
        gz = self._empty(batch) if need_noise_grad else None
        ws, n = self._workspace(batch, L.GRF_OP_BACKWARD)
        L.grf_backward(self.handle, int(seed) & (2 ** 64 - 1), _ptr(noise), batch, _ptr(th), _ptr(grad_out),
                       _ptr(gt), _ptr(gz), _ptr(ws), n, _stream())
        return gt, gz


class GRFSample(torch.autograd.Function):
    """phi = sampler(theta, z): differentiable in theta (sigma, length_scale,
    nu; [batch, 3] per field, or [3] shared by every field) and, when given,
    in the noise z ([batch, *dims]).

    apply(theta, plan, seed=0, noise=None, batch=None): the number of fields
    is noise.shape[0] when noise is given, else theta.shape[0] for a [batch, 3]
    theta; a shared [3] theta without noise needs `batch`.  Gradients come
    back on theta's (and the noise's) own device and dtype.

    The forward keeps only theta, the seed and the noise (if given); the
    backward recomputes the Fourier transform of the upstream gradient and
    regenerates the noise in the library (no spectrum is stored)."""

    @staticmethod
    def forward(ctx, theta, plan, seed=0, noise=None, batch=None):
        if theta.dim() not in (1, 2) or theta.shape[-1] != 3:
            raise ValueError(f"theta must be [batch, 3] or [3], got {tuple(theta.shape)}")
        if noise is not None:
            nb = int(noise.shape[0])
        elif theta.dim() == 2:
            nb = int(theta.shape[0])
        elif batch is None:
            raise ValueError("a shared theta of shape [3] without noise needs batch=")
        else:
            nb = int(batch)
        if batch is not None and int(batch) != nb:
            raise ValueError(f"batch={batch} does not match the {nb} fields of theta / noise")
        if theta.dim() == 2 and theta.shape[0] != nb:
            raise ValueError(f"theta has {theta.shape[0]} rows for {nb} fields")
        theta_c = theta.detach().to(device=plan.device, dtype=torch.float64)
        if theta_c.dim() == 1:
            theta_c = theta_c.expand(nb, 3)
        theta_c = theta_c.contiguous()
        if noise is None:
            out = plan.sample(seed=seed, batch=nb, theta=theta_c)
        else:
            out = plan.sample_from_noise(noise.detach(), theta=theta_c)
        ctx.plan, ctx.seed = plan, seed
        ctx.theta_dim = theta.dim()
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        ctx.noise_device = noise.device if noise is not None else None
        ctx.noise_dtype = noise.dtype if noise is not None else None
        ctx.save_for_backward(theta_c, noise.detach() if noise is not None else None)
        ctx.has_noise = noise is not None
        return out

    @staticmethod
    def backward(ctx, g):
        theta_c, noise = ctx.saved_tensors
        need_z = ctx.has_noise and ctx.needs_input_grad[3]
        gt, gz = ctx.plan.backward(g, seed=ctx.seed, theta=theta_c, noise=noise, need_noise_grad=need_z)
        if ctx.theta_dim == 1:
            gt = gt.sum(0)
        gt = gt.to(device=ctx.theta_device, dtype=ctx.theta_dtype)
        if gz is not None:
            gz = gz.to(device=ctx.noise_device, dtype=ctx.noise_dtype)
        return gt, None, None, gz, None


class Batch:
    """Fields of different sizes and parameters (d = 2, one-FFT, float32)
    sampled together by one persistent launch (per-XCD queues of column and
    last-axis items, per-field readiness counters; two launches where one
    cannot reach all 8 XCDs) replayed from a hipGraph.

    fields: iterable of dicts with keys dims=(N_1, N_2), seed, and optionally
    lengths, cov ('gaussian' | 'matern' | 'exponential'), sigma, length_scale, nu.
    """

    def __init__(self, fields, device=None):
        descs = []
        for f in fields:
            d = L.grf_field_desc()
            d.dims[0], d.dims[1] = (int(v) for v in f["dims"])
            ls = f.get("lengths", (1.0, 1.0))
            d.lengths[0], d.lengths[1] = float(ls[0]), float(ls[1])
            d.cov_kind = COV_KINDS[f.get("cov", "matern")]
            d.sigma = float(f.get("sigma", 1.0))
            d.length_scale = float(f.get("length_scale", 0.1))
            d.nu = float(f.get("nu", 1.5))
            d.seed = int(f["seed"]) & (2 ** 64 - 1)
            descs.append(d)
        self.n = len(descs)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            self.handle = L.grf_batch_create(descs)
        self.offsets = L.grf_batch_offsets(self.handle, self.n)
        self.dims = [tuple(int(v) for v in f["dims"]) for f in fields]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.lib.grf_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    def empty(self):
        return torch.empty(self.offsets[-1], dtype=torch.float32, device=self.device)

    def sample(self, out=None, plain=False):
        """Flat float32 output; field f is out[offsets[f]:offsets[f+1]] viewed as dims[f]."""
        out = self._out(out)
        f = L.grf_batch_sample_plain if plain else L.grf_batch_sample
        f(self.handle, _ptr(out), _stream())
        return out

    def _out(self, out):
        if out is None:
            return self.empty()
        return _check("out", out, (self.offsets[-1],), torch.float32, self.device)

    def tune(self, out=None):
        out = self._out(out)
        L.grf_batch_tune(self.handle, _ptr(out), _stream())

    def info(self):
        """(launches per sample: 1 or 2, row items whose wait gave up in the last sample)."""
        return L.grf_batch_info(self.handle)

    def field(self, out, f):
        return out[self.offsets[f]:self.offsets[f + 1]].view(self.dims[f])
