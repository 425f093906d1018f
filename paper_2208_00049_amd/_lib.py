"""ctypes loader for libnfft.so (argument marshalling only).

Raises ``RuntimeError`` when the shared library has not been built: there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfft.so")

# names and status codes of include/nfft.h
NFFT_OK = 0
NFFT_ERR_ARG = -1
NFFT_ERR_UNSUPPORTED = -2
NFFT_ERR_NOMEM = -3
NFFT_ERR_HIP = -4
NFFT_ERR_NODES = -5
NFFT_ERR_SCRATCH = -6
NOALLOC_SCRATCH_BYTES = 64 << 20  # NFFT_NOALLOC_SCRATCH_BYTES
NFFT_C64 = 0
NFFT_C128 = 1
NFFT_WINDOW_POLY = 0
NFFT_WINDOW_DIRECT = 1
NFFT_WINDOW_TENSOR = 2
NFFT_WINDOW_LINEAR = 3
NFFT_WINDOW_FULL = 4
WINDOWS = {"poly": NFFT_WINDOW_POLY, "direct": NFFT_WINDOW_DIRECT, "tensor": NFFT_WINDOW_TENSOR,
           "linear": NFFT_WINDOW_LINEAR, "full": NFFT_WINDOW_FULL}

EXPORTS = ["nfft_plan_create", "nfft_plan_create_ex", "nfft_plan_destroy", "nfft_forward",
           "nfft_adjoint", "nfft_resample_forward", "nfft_resample_adjoint", "nfft_fft_grid",
           "nfft_plan_info", "nfft_plan_grid", "nfft_plan_set_timing", "nfft_plan_timing",
           "nfft_plan_bench_stage", "nfft_forward_many", "nfft_adjoint_many",
           "nfft_batch_create", "nfft_batch_forward", "nfft_batch_adjoint", "nfft_batch_destroy",
           "nfft_plan_create_tuned", "nfft_forward_deriv", "nfft_node_grad", "nfft_strerror",
           "nfft_plan_window_peak", "nfft_calibrate_lds", "nfft_forward_many_noalloc",
           "nfft_plan_spread", "nfft_batch_info"]
SPREAD = {"auto": 0, "tiled": 1, "sweep": 2}
NFFT_NUM_STAGES = 8
LDS_OPS = {"ds_add_u32": 0, "ds_add_u64": 1, "ds_add_f32": 2, "ds_add_f64": 3,
           "ds_write_b64": 4, "rmw_b64": 5, "ds_read_b64": 6, "ds_read_b128": 7}
STAGES = ["fwd_deconv_fft_last", "fwd_fft_axis1", "fwd_fft_axis0", "interp", "spread",
          "adj_fft_axis0", "adj_fft_axis1", "adj_fft_last_deconv"]


class Options(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int * 4), ("window", ctypes.c_int),
                ("max_block_nodes", ctypes.c_int), ("wide", ctypes.c_int),
                ("spread", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class NfftError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, strerror(code), code))


_lib = None


def load():
    """Load libnfft.so once and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libnfft.so is not built (%s); run paper_2208_00049_amd/build.py "
                           "or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    plan_p = ctypes.POINTER(ctypes.c_void_p)
    lib.nfft_plan_create.argtypes = [plan_p, ctypes.c_int, i64p, ctypes.c_int64, vp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, vp]
    lib.nfft_plan_create_ex.argtypes = [plan_p, ctypes.c_int, i64p, ctypes.c_int64, vp,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(Options), vp]
    lib.nfft_plan_destroy.argtypes = [vp]
    lib.nfft_forward.argtypes = [vp, vp, vp, vp]
    lib.nfft_adjoint.argtypes = [vp, vp, vp, vp]
    lib.nfft_resample_forward.argtypes = [vp, vp, vp, vp]
    lib.nfft_resample_adjoint.argtypes = [vp, vp, vp, vp]
    lib.nfft_fft_grid.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.nfft_plan_info.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int)]
    lib.nfft_plan_grid.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p)]
    lib.nfft_plan_window_peak.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nfft_plan_spread.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.nfft_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.nfft_plan_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nfft_plan_bench_stage.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.nfft_forward_many.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.nfft_adjoint_many.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.nfft_forward_many_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.nfft_batch_create.argtypes = [plan_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_int]
    lib.nfft_batch_forward.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), vp]
    lib.nfft_batch_adjoint.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), vp]
    lib.nfft_batch_destroy.argtypes = [vp]
    lib.nfft_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]
    lib.nfft_plan_create_tuned.argtypes = [plan_p, ctypes.c_int, i64p, ctypes.c_int64, vp,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(Options), ctypes.c_int, vp,
                                           ctypes.POINTER(ctypes.c_double)]
    lib.nfft_forward_deriv.argtypes = [vp, vp, vp, vp]
    lib.nfft_node_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.nfft_calibrate_lds.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                       ctypes.POINTER(ctypes.c_double)]
    lib.nfft_strerror.argtypes = [ctypes.c_int]
    lib.nfft_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "nfft_strerror":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().nfft_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != NFFT_OK:
        raise NfftError(code, where)
