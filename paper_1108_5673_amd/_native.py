"""ctypes declarations of the C ABI in include/pwa.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIBRARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpwa.so")

PWA_OK = 0
PWA_WARN_DEGENERATE = 1
PWA_ERR_INVALID = -1
PWA_ERR_OOM = -2
PWA_ERR_DEVICE = -3
PWA_ERR_NO_DEVICE = -4
PWA_ERR_NONFINITE_INPUT = -5

PWA_FORM_TABLE = 1
PWA_FORM_AMPLITUDE = 2
PWA_INPUT_IS_TABLE = 4
PWA_PRECISION_FP64_PLAIN = 8
PWA_DATA_COMPLEX128 = 16
PWA_MC_COMPLEX128 = 32
PWA_PRECISION_FP64_FUSED = 64
PWA_FORM_AMPLITUDE_BF16 = 128
PWA_FORM_AMPLITUDE_FP16 = 256

PWA_MAX_WAVES_TABLE = 64
PWA_MAX_WAVES_AMPLITUDE = 128
PWA_MAX_WAVES_MATRIX = 64

# every symbol include/pwa.h declares
EXPORTED = (
    "pwa_build_table", "pwa_nll", "pwa_nll_grad", "pwa_nll_batched", "pwa_free",
    "pwa_last_error", "pwa_model_info", "pwa_copy_table", "pwa_copy_mc_matrix",
    "pwa_set_mc_matrix", "pwa_set_timing", "pwa_get_timing", "pwa_build_timing",
    "pwa_lbfgs_default_options", "pwa_lbfgs_minimize", "pwa_fit_lbfgs", "pwa_nll_grad_hess",
    "pwa_newton_minimize", "pwa_fit_fumili", "pwa_get_amplitude_shape",
    "pwa_set_amplitude_shape", "pwa_tune_amplitude_shape", "pwa_nll_async",
    "pwa_nll_grad_async", "pwa_read_ceiling", "pwa_nll_batched_noalloc",
)

PWA_LBFGS_CONVERGED_GRADIENT = 0
PWA_LBFGS_CONVERGED_VALUE = 1
PWA_LBFGS_MAX_ITERATIONS = 2
PWA_LBFGS_LINE_SEARCH_FAILED = 3

# int (*)(void* ctx, const double* x, double* f, double* g)
OBJECTIVE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


# int (*)(void* ctx, const double* x, double* f, double* g, double* H)
OBJECTIVE_HESS = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double))


class LbfgsOptions(ctypes.Structure):
    _fields_ = [
        ("max_iterations", ctypes.c_int32),
        ("history", ctypes.c_int32),
        ("grad_tol", ctypes.c_double),
        ("rel_f_tol", ctypes.c_double),
        ("fixed_index", ctypes.c_int32),
    ]


class LbfgsResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("evaluations", ctypes.c_int32),
        ("f", ctypes.c_double),
        ("grad_norm", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_data", ctypes.c_int64),
        ("n_waves", ctypes.c_int32),
        ("n_packed", ctypes.c_int32),
        ("form", ctypes.c_uint32),
        ("stream_bytes", ctypes.c_int64),
        ("grid_blocks", ctypes.c_int32),
        ("compute_units", ctypes.c_int32),
    ]


class PWAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("pwa status %d: %s" % (status, message))
        self.status = status


_lib = None


def lib():
    """The loaded HIP library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError("the HIP library %s is not built; run "
                               "`python -m paper_1108_5673_amd.build`" % LIBRARY)
        _lib = _declare(ctypes.CDLL(LIBRARY))
    return _lib


def _declare(L):
    p, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    dp = ctypes.POINTER(ctypes.c_double)
    L.pwa_build_table.argtypes = [p, i64, i32, p, i64, i64, u32, p, ctypes.POINTER(p)]
    L.pwa_nll.argtypes = [p, p, dp, p]
    L.pwa_nll_grad.argtypes = [p, p, dp, p, p]
    L.pwa_nll_grad_hess.argtypes = [p, p, dp, p, p, p]
    L.pwa_nll_batched.argtypes = [p, i32, p, p, p, p, p]
    L.pwa_free.argtypes = [p]
    L.pwa_free.restype = None
    L.pwa_last_error.argtypes = []
    L.pwa_last_error.restype = ctypes.c_char_p
    L.pwa_model_info.argtypes = [p, ctypes.POINTER(Info)]
    L.pwa_copy_table.argtypes = [p, p, p]
    L.pwa_copy_mc_matrix.argtypes = [p, p, p]
    L.pwa_set_mc_matrix.argtypes = [p, p, p]
    L.pwa_set_timing.argtypes = [p, ctypes.c_int]
    L.pwa_nll_async.argtypes = [p, p, p, p]
    L.pwa_read_ceiling.argtypes = [p, ctypes.c_int32, p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.pwa_nll_grad_async.argtypes = [p, p, p, p]
    L.pwa_nll_batched_noalloc.argtypes = [p, i32, p, p, p]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.pwa_get_amplitude_shape.argtypes = [p, i32p, i32p]
    L.pwa_set_amplitude_shape.argtypes = [p, ctypes.c_int32, ctypes.c_int32, p]
    L.pwa_tune_amplitude_shape.argtypes = [p, ctypes.c_int32, p, i32p, i32p]
    L.pwa_get_timing.argtypes = [p, dp, ctypes.POINTER(i64)]
    L.pwa_build_timing.argtypes = [p, dp, dp]
    L.pwa_lbfgs_default_options.argtypes = [ctypes.POINTER(LbfgsOptions)]
    L.pwa_lbfgs_default_options.restype = None
    L.pwa_lbfgs_minimize.argtypes = [i32, dp, OBJECTIVE, p, ctypes.POINTER(LbfgsOptions),
                                     ctypes.POINTER(LbfgsResult)]
    L.pwa_fit_lbfgs.argtypes = [p, dp, ctypes.POINTER(LbfgsOptions), ctypes.POINTER(LbfgsResult), p]
    L.pwa_newton_minimize.argtypes = [i32, dp, OBJECTIVE_HESS, p, ctypes.POINTER(LbfgsOptions),
                                      ctypes.POINTER(LbfgsResult)]
    L.pwa_fit_fumili.argtypes = [p, dp, ctypes.POINTER(LbfgsOptions), ctypes.POINTER(LbfgsResult), p]
    for name in EXPORTED:
        if name not in ("pwa_free", "pwa_last_error", "pwa_lbfgs_default_options"):
            getattr(L, name).restype = ctypes.c_int
    return L


def last_error() -> str:
    msg = lib().pwa_last_error()
    return msg.decode() if msg else ""


def check(status: int) -> int:
    """Raise PWAError for errors; pass OK and warnings through."""
    if status < 0:
        raise PWAError(status, last_error())
    return status
