"""The C ABI library loads and exports every declared symbol; host-side
validation rejects bad descriptors before any device work.  CPU only: nothing
here initialises a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grf.h")
LIB = os.path.join(ROOT, "paper_1105_2737_amd", "libgrf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgrf.so not built")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(grf_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_binding_exports():
    from paper_1105_2737_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


def _desc(**kw):
    from paper_1105_2737_amd import _lib as L
    d = L.grf_plan_desc()
    d.ndim, d.alg, d.dtype, d.cov_kind = 2, L.GRF_ALG_ONE_FFT, L.GRF_F32, L.GRF_COV_MATERN
    d.dims[0], d.dims[1] = 64, 64
    d.lengths[0] = d.lengths[1] = d.lengths[2] = 1.0
    d.sigma, d.length_scale, d.nu = 1.0, 0.1, 1.5
    for k, v in kw.items():
        if k == "dims":
            for i, n in enumerate(v):
                d.dims[i] = n
        elif k == "lengths":
            for i, n in enumerate(v):
                d.lengths[i] = n
        elif k == "bc":
            for i, n in enumerate(v):
                d.bc[i] = n
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(dims=(63, 64)), -1),            # odd N (the paper requires even N_i)
    (dict(dims=(64, 14)), -1),            # prime factor 7
    (dict(dims=(0, 64)), -1),
    (dict(sigma=0.0), -1),
    (dict(length_scale=-1.0), -1),
    (dict(nu=0.0), -1),
    (dict(lengths=(1.0, 0.0)), -1),
    (dict(alg=3), -1),
    (dict(dtype=7), -1),
    (dict(cov_kind=9), -1),
    (dict(ndim=4), -1),
    (dict(ndim=0), -1),
    (dict(dims=(8192, 64)), -4),          # leading axis above the runtime-radix limit (4096)
    (dict(dims=(64, 32768)), -4),         # last axis above its limit (16384)
    (dict(ndim=1, dims=(14,)), -1),
    (dict(ndim=1, dims=(32768,)), -4),
    (dict(dims=(80, 64), bc=(1, 1)), -4),            # reflecting boundaries: listed lengths only
    (dict(dims=(64, 90), draw_order=1), -4),         # recursive draw order: listed lengths only
    (dict(cov_kind=3, m=0.0, k=1, l=1, n=1), -1),   # the family of Section 4 needs m > 0
    (dict(cov_kind=3, m=1.0, k=0, l=1, n=1), -1),   # and k, l, n >= 1
    (dict(cov_kind=3, m=1.0, k=1, l=1, n=65), -1),
    (dict(cov_kind=4), -1),                          # tabulated density without a table
    (dict(cov_kind=5), -1),
    (dict(bc=(3, 3)), -1),                           # unknown boundary condition
    (dict(bc=(-1, 1)), -1),
    (dict(bc=(1, 0)), -4),                           # periodic and reflecting axes mixed
    (dict(ndim=3, dims=(16, 16, 16), bc=(2, 0, 2)), -4),
    (dict(alg=1, bc=(1, 1)), -4),                    # reflecting: one-transform method only
    (dict(draw_order=2), -1),                        # unknown draw order
    (dict(draw_order=1, alg=1), -4),                 # recursive order: one-FFT algorithm only
    (dict(draw_order=1, bc=(2, 2)), -4),             # and periodic axes
])
def test_invalid_descriptors_are_rejected_on_the_host(kw, status):
    from paper_1105_2737_amd import _lib as L
    h = ctypes.c_void_p()
    st = L.lib.grf_plan_create(ctypes.byref(_desc(**kw)), ctypes.byref(h))
    assert st == status, L.grf_last_error()
    assert not h.value
    assert L.grf_last_error()


def test_null_arguments():
    from paper_1105_2737_amd import _lib as L
    assert L.lib.grf_plan_create(None, None) == L.GRF_EINVAL
    assert L.lib.grf_plan_destroy(None) == L.GRF_OK
    n = ctypes.c_size_t()
    assert L.lib.grf_workspace_size(None, 1, 0, ctypes.byref(n)) == L.GRF_EINVAL
    assert L.lib.grf_sample(None, 0, 1, None, None, None, 0, None) == L.GRF_EINVAL
    assert L.lib.grf_backward(None, 0, None, 1, None, None, None, None, None, 0, None) == L.GRF_EINVAL
    assert L.lib.grf_covariance(None, 0, 1, None, None, 0, None) == L.GRF_EINVAL
    assert L.lib.grf_debug_philox(0, None, -1, None, None) == L.GRF_EINVAL
    assert L.lib.grf_debug_philox(0, None, 0, None, None) == L.GRF_OK
    assert L.grf_version().startswith("grf-mi355x")


@pytest.mark.parametrize("dims,status", [((64, 63), -1), ((64, 14), -1), ((2048, 64), -4), ((64, 2048), -4),
                                         ((4, 64), -4)])
def test_batch_descriptors_rejected_on_the_host(dims, status):
    from paper_1105_2737_amd import _lib as L
    d = L.grf_field_desc()
    d.dims[0], d.dims[1] = dims
    d.lengths[0] = d.lengths[1] = 1.0
    d.cov_kind, d.sigma, d.length_scale, d.nu, d.seed = 1, 1.0, 0.1, 1.5, 0
    arr = (L.grf_field_desc * 1)(d)
    h = ctypes.c_void_p()
    assert L.lib.grf_batch_create(arr, 1, ctypes.byref(h)) == status
    assert not h.value
    assert L.lib.grf_batch_create(arr, 0, ctypes.byref(h)) == L.GRF_EINVAL
    assert L.lib.grf_batch_destroy(None) == L.GRF_OK
