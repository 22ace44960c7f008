"""ctypes declarations of libtrinv's C ABI (include/trinv.h).

The shared library is built in-tree by ``paper_2307_07611_amd/build.py``.
There is no fallback: if the library is missing, loading raises.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrinv.so")

F64, F32, BF16_REFINE, F16_REFINE = 0, 1, 2, 3
MODES = {"f64": F64, "f32": F32, "bf16_refine": BF16_REFINE, "f16_refine": F16_REFINE}

OK, ERR_ARG, ERR_SINGULAR, ERR_NONFINITE, ERR_NOT_CONVERGED, ERR_HIP, ERR_UNSUPPORTED, ERR_WORKSPACE = range(8)

RESID_AUTO, RESID_SPLIT, RESID_FP64 = 0, 1, 2
RESID = {"auto": RESID_AUTO, "split": RESID_SPLIT, "fp64": RESID_FP64}

EXPORTS = [
    "trinv_default_opts", "trinv_status_string", "trinv_workspace_bytes", "trinv_tril_inverse",
    "trinv_batched_workspace_bytes", "trinv_tril_inverse_batched", "trinv_batched_autotune",
    "trinv_batched_set_config", "trinv_batched_get_config", "trinv_tril_inverse_batched_noalloc",
    "trinv_backward_workspace_bytes",
    "trinv_tril_inverse_backward", "trinv_factored_workspace_bytes", "trinv_factored_inverse",
    "trinv_residual_workspace_bytes", "trinv_residual", "trinv_refine_residual_workspace_bytes",
    "trinv_refine_residual", "trinv_profile_enable", "trinv_profile_read",
    "trinv_profile_select",
    "trinv_skul_workspace_bytes", "trinv_skul", "trinv_sqr_workspace_bytes", "trinv_sqr",
    "trinv_brsi_workspace_bytes", "trinv_brsi",
]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("unit_diag", ctypes.c_int32), ("upper", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("blocking", ctypes.c_int32),
                ("check", ctypes.c_int32), ("beta", ctypes.c_int32), ("resid", ctypes.c_int32)]


class BatchedConfig(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("ms", ctypes.c_float),
                ("tile", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("rel_residual", ctypes.c_double), ("resid_error_est", ctypes.c_double),
                ("resid_error_bound", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("first_bad_index", ctypes.c_int64)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


def load():
    """Load libtrinv.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} not found: build it with paper_2307_07611_amd/build.py; "
                      "there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    lib.trinv_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.trinv_default_opts.restype = None
    lib.trinv_status_string.argtypes = [ctypes.c_int]
    lib.trinv_status_string.restype = ctypes.c_char_p
    lib.trinv_workspace_bytes.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(Opts)]
    lib.trinv_workspace_bytes.restype = _sz
    lib.trinv_tril_inverse.argtypes = [ctypes.c_int, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _sz,
                                       _vp, ctypes.POINTER(Info)]
    lib.trinv_tril_inverse.restype = ctypes.c_int
    lib.trinv_batched_workspace_bytes.argtypes = [ctypes.c_int, _i64, _vp, ctypes.POINTER(Opts)]
    lib.trinv_batched_workspace_bytes.restype = _sz
    lib.trinv_tril_inverse_batched.argtypes = [ctypes.c_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                               ctypes.POINTER(Opts), _vp, _sz, _vp]
    lib.trinv_tril_inverse_batched.restype = ctypes.c_int
    lib.trinv_tril_inverse_batched_noalloc.argtypes = [ctypes.c_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                       ctypes.POINTER(Opts), _vp]
    lib.trinv_tril_inverse_batched_noalloc.restype = ctypes.c_int
    lib.trinv_batched_autotune.argtypes = lib.trinv_tril_inverse_batched.argtypes + [ctypes.POINTER(BatchedConfig)]
    lib.trinv_batched_autotune.restype = ctypes.c_int
    lib.trinv_batched_set_config.argtypes = [ctypes.c_int, _i64, _vp, ctypes.POINTER(BatchedConfig)]
    lib.trinv_batched_set_config.restype = ctypes.c_int
    lib.trinv_batched_get_config.argtypes = [ctypes.c_int, _i64, _vp, ctypes.POINTER(BatchedConfig)]
    lib.trinv_batched_get_config.restype = ctypes.c_int
    lib.trinv_backward_workspace_bytes.argtypes = [ctypes.c_int, _i64, _i64]
    lib.trinv_backward_workspace_bytes.restype = _sz
    lib.trinv_tril_inverse_backward.argtypes = [ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _i64, _vp, _sz, _vp]
    lib.trinv_tril_inverse_backward.restype = ctypes.c_int
    lib.trinv_factored_workspace_bytes.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(Opts)]
    lib.trinv_factored_workspace_bytes.restype = _sz
    lib.trinv_factored_inverse.argtypes = [ctypes.c_int, _i64, _vp, _i64, _i32, _vp, _i64, _i32, _vp, _i64, _vp,
                                           _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _sz, _vp,
                                           ctypes.POINTER(Info)]
    lib.trinv_factored_inverse.restype = ctypes.c_int
    lib.trinv_skul_workspace_bytes.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(Opts)]
    lib.trinv_skul_workspace_bytes.restype = _sz
    lib.trinv_skul.argtypes = [ctypes.c_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz,
                               _vp, ctypes.POINTER(Info)]
    lib.trinv_skul.restype = ctypes.c_int
    lib.trinv_sqr_workspace_bytes.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(Opts)]
    lib.trinv_sqr_workspace_bytes.restype = _sz
    lib.trinv_sqr.argtypes = [ctypes.c_int, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz, _vp,
                              ctypes.POINTER(Info)]
    lib.trinv_sqr.restype = ctypes.c_int
    lib.trinv_brsi_workspace_bytes.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(Opts)]
    lib.trinv_brsi_workspace_bytes.restype = _sz
    lib.trinv_brsi.argtypes = [ctypes.c_int, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _sz, _vp,
                               ctypes.POINTER(Info)]
    lib.trinv_brsi.restype = ctypes.c_int
    lib.trinv_residual_workspace_bytes.argtypes = [ctypes.c_int, _i64]
    lib.trinv_residual_workspace_bytes.restype = _sz
    lib.trinv_residual.argtypes = [ctypes.c_int, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.trinv_residual.restype = ctypes.c_int
    lib.trinv_refine_residual_workspace_bytes.argtypes = [ctypes.c_int, _i64]
    lib.trinv_refine_residual_workspace_bytes.restype = _sz
    lib.trinv_refine_residual.argtypes = [ctypes.c_int, _i64, _vp, _i64, _vp, _i64, _i32, _vp, _i64, _vp, _sz, _vp,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.trinv_refine_residual.restype = ctypes.c_int
    lib.trinv_profile_enable.argtypes = [ctypes.c_int]
    lib.trinv_profile_enable.restype = ctypes.c_int
    lib.trinv_profile_read.argtypes = [ctypes.POINTER(ProfileEntry), ctypes.c_int]
    lib.trinv_profile_read.restype = ctypes.c_int
    lib.trinv_profile_select.argtypes = [ctypes.c_char_p]
    lib.trinv_profile_select.restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().trinv_status_string(code).decode()


class TrinvError(RuntimeError):
    def __init__(self, code: int, where: str, info=None):
        super().__init__(f"{where}: {status_string(code)} (status {code})")
        self.code = code
        self.info = info
