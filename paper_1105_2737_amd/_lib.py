"""ctypes binding of libgrf.so: the C ABI of include/grf.h under the same
names.  Argument marshalling only; every step of the sampler runs in the HIP
library.  Importing this module fails loudly if the library is not built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrf.so")

GRF_OK, GRF_EINVAL, GRF_ENOMEM, GRF_EDEVICE, GRF_EUNSUPPORTED = 0, -1, -2, -3, -4
GRF_ALG_TWO_FFT, GRF_ALG_ONE_FFT = 1, 2
GRF_F32, GRF_F64 = 0, 1
GRF_COV_GAUSSIAN, GRF_COV_MATERN, GRF_COV_EXPONENTIAL, GRF_COV_PAPER, GRF_COV_TABULATED = 0, 1, 2, 3, 4
GRF_OP_SAMPLE, GRF_OP_BACKWARD, GRF_OP_COVARIANCE = 0, 1, 2
GRF_PASS_COL_GEN_INV, GRF_PASS_COL_LOAD_INV, GRF_PASS_COL_LOAD_FWD = 0, 1, 2
GRF_PASS_COL_FILTER, GRF_PASS_COL_GRAD, GRF_PASS_ROW_C2R, GRF_PASS_ROW_R2C_GEN, GRF_PASS_ROW_R2C_LOAD = 3, 4, 5, 6, 7
GRF_PASS_ROW_GEN_C2R = 8
GRF_PASS_R2R_COL_GEN, GRF_PASS_R2R_COL_LOAD, GRF_PASS_R2R_ROW_LOAD, GRF_PASS_R2R_ROW_GEN = 9, 10, 11, 12
GRF_PASS_COL_SEQ_INV = 13
GRF_PASS_SPEC_FILTER = 14
GRF_BC_PERIODIC, GRF_BC_NEUMANN, GRF_BC_DIRICHLET = 0, 1, 2
GRF_DRAW_COUNTER, GRF_DRAW_RECURSIVE = 0, 1
GRF_NOALLOC_MAX_FIELDS = 65536

STATUS_NAMES = {0: "GRF_OK", -1: "GRF_EINVAL", -2: "GRF_ENOMEM", -3: "GRF_EDEVICE", -4: "GRF_EUNSUPPORTED"}

# every symbol include/grf.h declares
EXPORTS = ["grf_plan_create", "grf_plan_destroy", "grf_workspace_size", "grf_sample", "grf_sample_noalloc",
           "grf_sample_stage_count", "grf_sample_stage", "grf_sample_stage_info", "grf_sample_from_noise", "grf_noise", "grf_backward", "grf_debug_philox",
           "grf_debug_spectrum",
           "grf_covariance", "grf_batch_create", "grf_batch_offsets", "grf_batch_sample", "grf_batch_sample_plain",
           "grf_batch_tune", "grf_batch_destroy", "grf_last_error", "grf_version", "grf_plan_tune",
           "grf_plan_tune_choice", "grf_batch_info"]


class grf_plan_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("alg", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("cov_kind", ctypes.c_int32), ("dims", ctypes.c_int64 * 3), ("lengths", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("length_scale", ctypes.c_double), ("nu", ctypes.c_double),
                ("m", ctypes.c_double), ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("spectrum", ctypes.c_void_p), ("bc", ctypes.c_int32 * 3),
                ("draw_order", ctypes.c_int32)]


class grf_field_desc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 2), ("lengths", ctypes.c_double * 2), ("cov_kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("sigma", ctypes.c_double), ("length_scale", ctypes.c_double),
                ("nu", ctypes.c_double), ("seed", ctypes.c_uint64)]


class GRFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1105_2737_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, c64, u64, sz, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int32
    sig = {
        "grf_plan_create": (ctypes.c_int, [ctypes.POINTER(grf_plan_desc), ctypes.POINTER(vp)]),
        "grf_plan_destroy": (ctypes.c_int, [vp]),
        "grf_workspace_size": (ctypes.c_int, [vp, c64, i32, ctypes.POINTER(sz)]),
        "grf_sample": (ctypes.c_int, [vp, u64, c64, vp, vp, vp, sz, vp]),
        "grf_sample_noalloc": (ctypes.c_int, [vp, u64, c64, vp, vp, vp]),
        "grf_sample_stage_count": (ctypes.c_int, [vp, c64, ctypes.POINTER(i32)]),
        "grf_sample_stage": (ctypes.c_int, [vp, i32, u64, c64, vp, vp, vp, sz, vp]),
        "grf_sample_stage_info": (ctypes.c_int, [vp, c64, i32, ctypes.POINTER(i32), ctypes.POINTER(c64),
                                                 ctypes.POINTER(c64)]),
        "grf_sample_from_noise": (ctypes.c_int, [vp, vp, c64, vp, vp, vp, sz, vp]),
        "grf_noise": (ctypes.c_int, [vp, u64, c64, vp, vp]),
        "grf_backward": (ctypes.c_int, [vp, u64, vp, c64, vp, vp, vp, vp, vp, sz, vp]),
        "grf_debug_philox": (ctypes.c_int, [u64, vp, c64, vp, vp]),
        "grf_debug_spectrum": (ctypes.c_int, [vp, u64, c64, vp, vp]),
        "grf_covariance": (ctypes.c_int, [vp, u64, c64, vp, vp, sz, vp]),
        "grf_batch_create": (ctypes.c_int, [ctypes.POINTER(grf_field_desc), c64, ctypes.POINTER(vp)]),
        "grf_batch_offsets": (ctypes.c_int, [vp, ctypes.POINTER(c64)]),
        "grf_batch_sample": (ctypes.c_int, [vp, vp, vp]),
        "grf_batch_sample_plain": (ctypes.c_int, [vp, vp, vp]),
        "grf_batch_tune": (ctypes.c_int, [vp, vp, vp]),
        "grf_batch_destroy": (ctypes.c_int, [vp]),
        "grf_batch_info": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "grf_plan_tune": (ctypes.c_int, [vp, c64, vp, vp]),
        "grf_plan_tune_choice": (ctypes.c_int, [vp, i32, c64, ctypes.c_char_p, sz]),
        "grf_last_error": (ctypes.c_char_p, []),
        "grf_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(status):
    if status != GRF_OK:
        raise GRFError(status, lib.grf_last_error().decode())
    return status


# ---- same-name wrappers (raise GRFError on a non-OK status) ----------------

def grf_plan_create(desc):
    h = ctypes.c_void_p()
    check(lib.grf_plan_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def grf_plan_destroy(plan):
    return check(lib.grf_plan_destroy(plan))


def grf_workspace_size(plan, batch, op):
    n = ctypes.c_size_t()
    check(lib.grf_workspace_size(plan, batch, op, ctypes.byref(n)))
    return n.value


def grf_sample(plan, seed, batch, theta, out, workspace, workspace_bytes, stream):
    return check(lib.grf_sample(plan, seed, batch, theta, out, workspace, workspace_bytes, stream))


def grf_sample_noalloc(plan, seed, batch, theta, out, stream):
    return check(lib.grf_sample_noalloc(plan, seed, batch, theta, out, stream))


def grf_sample_stage_count(plan, batch):
    n = ctypes.c_int32()
    check(lib.grf_sample_stage_count(plan, batch, ctypes.byref(n)))
    return n.value


def grf_sample_stage(plan, stage, seed, batch, theta, out, workspace, workspace_bytes, stream):
    return check(lib.grf_sample_stage(plan, stage, seed, batch, theta, out, workspace, workspace_bytes, stream))


def grf_sample_stage_info(plan, batch, stage):
    """(kind, first, count) of launch `stage` for a batch of `batch` fields."""
    kind, first, count = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    check(lib.grf_sample_stage_info(plan, batch, stage, ctypes.byref(kind), ctypes.byref(first), ctypes.byref(count)))
    return kind.value, first.value, count.value


def grf_sample_from_noise(plan, noise, batch, theta, out, workspace, workspace_bytes, stream):
    return check(lib.grf_sample_from_noise(plan, noise, batch, theta, out, workspace, workspace_bytes, stream))


def grf_noise(plan, seed, batch, out, stream):
    return check(lib.grf_noise(plan, seed, batch, out, stream))


def grf_backward(plan, seed, noise, batch, theta, grad_out, grad_theta, grad_noise, workspace,
                 workspace_bytes, stream):
    return check(lib.grf_backward(plan, seed, noise, batch, theta, grad_out, grad_theta, grad_noise,
                                  workspace, workspace_bytes, stream))


def grf_covariance(plan, seed, nsamples, cov, workspace, workspace_bytes, stream):
    return check(lib.grf_covariance(plan, seed, nsamples, cov, workspace, workspace_bytes, stream))


def grf_debug_philox(seed, counters, n, out, stream):
    return check(lib.grf_debug_philox(seed, counters, n, out, stream))


def grf_debug_spectrum(plan, seed, batch, out, stream):
    return check(lib.grf_debug_spectrum(plan, seed, batch, out, stream))


def grf_batch_create(fields):
    n = len(fields)
    arr = (grf_field_desc * n)(*fields)
    h = ctypes.c_void_p()
    check(lib.grf_batch_create(arr, n, ctypes.byref(h)))
    return h


def grf_batch_offsets(batch, nfields):
    arr = (ctypes.c_int64 * (nfields + 1))()
    check(lib.grf_batch_offsets(batch, arr))
    return list(arr)


def grf_batch_sample(batch, out, stream):
    return check(lib.grf_batch_sample(batch, out, stream))


def grf_batch_sample_plain(batch, out, stream):
    return check(lib.grf_batch_sample_plain(batch, out, stream))


def grf_batch_tune(batch, out, stream):
    return check(lib.grf_batch_tune(batch, out, stream))


def grf_batch_info(batch):
    n, e = ctypes.c_int32(), ctypes.c_int32()
    check(lib.grf_batch_info(batch, ctypes.byref(n), ctypes.byref(e)))
    return n.value, e.value


def grf_batch_destroy(batch):
    return check(lib.grf_batch_destroy(batch))


def grf_plan_tune(plan, batch, out, stream):
    return check(lib.grf_plan_tune(plan, batch, out, stream))


def grf_plan_tune_choice(plan, pass_, length):
    buf = ctypes.create_string_buffer(128)
    check(lib.grf_plan_tune_choice(plan, pass_, length, buf, 128))
    return buf.value.decode()


def grf_last_error():
    return lib.grf_last_error().decode()


def grf_version():
    return lib.grf_version().decode()
