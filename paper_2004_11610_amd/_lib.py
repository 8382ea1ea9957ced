"""ctypes declarations of the C ABI in include/spt.h (argument marshalling only)."""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspt.so")

SPT_OK = 0
NOALLOC_MAX_BYTES = 32 << 20  # SPT_NOALLOC_MAX_BYTES
ERRORS = {-1: "SPT_E_INVALID_ARG", -2: "SPT_E_NOT_PRECOMPUTED", -3: "SPT_E_HIP",
          -4: "SPT_E_OOM", -5: "SPT_E_UNSUPPORTED", -6: "SPT_E_NUMERIC"}


class SptParams(ctypes.Structure):
    _fields_ = [("alpha", c_double), ("beta", c_double), ("eps2", c_double),
                ("mode", c_int32), ("unweighted", c_int32), ("precisions", c_uint32),
                ("min_block", c_int32), ("exact_fft_len", c_int32), ("executor", c_int32),
                ("panel_rows", c_int64), ("nodes", POINTER(c_double)), ("power", c_int32),
                ("trig_conv_q", c_int32), ("eta", c_double), ("period", c_double),
                ("reduced_fft", c_int32)]


class SptPlanInfo(ctypes.Structure):
    _fields_ = [("family", c_int32), ("mode", c_int32), ("n_blocks", c_int32),
                ("tail", c_int32), ("N", c_int64), ("eps1", c_double), ("eps2", c_double),
                ("zeta", c_double), ("precomputed", c_int32), ("max_band", c_int32),
                ("nnz", c_int64), ("stored", c_int64), ("matrix_bytes_f64", c_int64),
                ("matrix_bytes_f32", c_int64), ("max_abs", c_double * 16),
                ("kappa", c_double), ("nnz_blk", c_int64 * 16), ("window_lds", c_int64),
                ("window_cols", c_int64), ("window_chunked", c_int64),
                ("transposed_segment", c_int64), ("reduced_fft_f64", c_int64),
                ("is_complex", c_int64), ("reduced_fft_f32_err", c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


class SptTuning(ctypes.Structure):
    _fields_ = [("product", c_int32), ("window_rhs", c_int32), ("fft_batch", c_int32),
                ("fft_half", c_int32), ("inv_four", c_int32)]


class SptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load():
    """Load libspt.so; there is no fallback: the library must be built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libspt.so is not built (run `python -m paper_2004_11610_amd.build`)")
    lib = ctypes.CDLL(LIB_PATH)
    p_plan = POINTER(c_void_p)
    sig = {
        "spt_plan_create": [p_plan, c_int32, POINTER(SptParams), c_int64, c_double],
        "spt_plan_blocks": [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                            POINTER(c_int32), c_int32, POINTER(c_int32)],
        "spt_precompute": [c_void_p, c_void_p],
        "spt_execute": [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p],
        "spt_execute_transposed": [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p],
        "spt_execute_noalloc": [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p],
        "spt_execute_batched": [POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                POINTER(c_int64), c_int32, c_int32, c_void_p],
        "spt_plan_query": [c_void_p, POINTER(SptPlanInfo)],
        "spt_plan_set_exec_wait": [c_void_p, c_int64],
        "spt_set_allocator": [ALLOC_FN, FREE_FN, c_void_p],
        "spt_plan_set_tuning": [c_void_p, POINTER(SptTuning)],
        "spt_plan_get_tuning": [c_void_p, POINTER(SptTuning)],
        "spt_autotune": [c_void_p, c_int64, c_int32, c_void_p, c_char_p, POINTER(SptTuning),
                         POINTER(c_double)],
        "spt_plan_nodes": [c_void_p, POINTER(c_double)],
        "spt_plan_compressed_rows": [c_void_p, c_int32, c_int64, c_int64, POINTER(c_double)],
        "spt_plan_destroy": [c_void_p],
        "spt_profile_begin": [],
        "spt_profile_end": [POINTER(c_double), POINTER(c_int64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.spt_last_error.argtypes = []
    lib.spt_last_error.restype = c_char_p
    lib.spt_version.argtypes = []
    lib.spt_version.restype = c_char_p
    _lib = lib
    return lib


def check(status):
    if status != SPT_OK:
        raise SptError(status, load().spt_last_error().decode())
    return status
