"""ctypes declarations of the C ABI in include/precode.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libprecode.so")

# return codes
OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE = 0, -1, -2, -3, -4
# status flags
ST_OK, ST_FAIL, ST_FP64 = 0, 1, 2
# enums
ZF, WF = 0, 1
ARCH_PD, ARCH_FD = 0, 1
PREC_FP32, PREC_SPLIT_FP16, PREC_SPLIT_BF16, PREC_FP64 = 0, 1, 2, 3
IMPL_AUTO, IMPL_FUSED, IMPL_PLAIN = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [
        ("power", ctypes.c_float),
        ("Es", ctypes.c_float),
        ("tau", ctypes.c_float),
        ("precision", ctypes.c_int),
        ("refine_steps", ctypes.c_int),
        ("fp64_ratio", ctypes.c_float),
        ("impl", ctypes.c_int),
        ("cluster_tau", ctypes.POINTER(ctypes.c_float)),
        ("cluster_power", ctypes.POINTER(ctypes.c_float)),
    ]


class Job(ctypes.Structure):
    _fields_ = [
        ("arch", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("B", ctypes.c_int),
        ("U", ctypes.c_int),
        ("n_sc", ctypes.c_int),
        ("K", ctypes.c_int),
        ("C", ctypes.c_int),
        ("cluster_sizes", ctypes.POINTER(ctypes.c_int)),
        ("rho", ctypes.c_float),
        ("power", ctypes.c_float),
        ("Es", ctypes.c_float),
        ("tau", ctypes.c_float),
        ("H", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("scale", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class ServeJob(ctypes.Structure):
    _fields_ = [("job", Job), ("arrival_s", ctypes.c_double), ("symbol_period_s", ctypes.c_double)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int), ("n_streams", ctypes.c_int), ("precision", ctypes.c_int),
                ("slab_bytes", ctypes.c_size_t), ("impl", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("jobs_done", ctypes.c_int), ("peak_active", ctypes.c_int), ("symbols_done", ctypes.c_longlong),
                ("subcarrier_symbols_done", ctypes.c_longlong), ("wall_s", ctypes.c_double),
                ("throughput", ctypes.c_double), ("lat_p50_s", ctypes.c_double), ("lat_p99_s", ctypes.c_double),
                ("lat_max_s", ctypes.c_double), ("wait_p50_s", ctypes.c_double), ("wait_p99_s", ctypes.c_double),
                ("peak_bytes", ctypes.c_size_t)]


VP = ctypes.c_void_p
I = ctypes.c_int
F = ctypes.c_float
IP = ctypes.POINTER(ctypes.c_int)
SZ = ctypes.c_size_t

SIGNATURES = {
    "precode_params_init": (None, [ctypes.POINTER(Params)]),
    "precode_strerror": (ctypes.c_char_p, [I]),
    "precode_validate": (I, [I, F, IP, I, I, I, I, I, I, ctypes.POINTER(Params)]),
    "precode_ctx_create": (I, [I, SZ, ctypes.POINTER(VP)]),
    "precode_ctx_destroy": (I, [VP]),
    "precode_ctx_bytes": (SZ, [VP]),
    "precode_ctx_last_impl": (I, [VP]),
    "precode_ctx_last_waves": (I, [VP]),
    "precode_pd": (I, [VP, VP, VP, F, IP, I, I, I, I, I, I, ctypes.POINTER(Params), VP, VP, VP, VP]),
    "precode_fd": (I, [VP, VP, VP, F, IP, I, I, I, I, I, I, ctypes.POINTER(Params), VP, VP, VP, VP]),
    "precode_pd_noalloc": (I, [VP, VP, VP, F, IP, I, I, I, I, I, I, ctypes.POINTER(Params), VP, VP, VP, VP]),
    "precode_central": (I, [VP, VP, VP, F, I, I, I, I, ctypes.POINTER(Params), VP, VP, VP, VP]),
    "precode_mrt": (I, [VP, VP, VP, IP, I, I, I, I, I, ctypes.POINTER(Params), VP, VP, VP, VP]),
    "precode_qam_map": (I, [VP, ctypes.c_longlong, I, VP, VP]),
    "precode_ue_receive": (I, [VP, VP, VP, F, VP, I, I, I, I, VP, VP]),
    "precode_ue_gain": (I, [VP, F, F, I, I, VP, VP]),
    "precode_qam_errors": (I, [VP, VP, ctypes.c_longlong, I, VP, VP, VP]),
    "precode_frame_prepare": (I, [VP, I, VP, F, IP, I, I, I, I, I, ctypes.POINTER(Params),
                                  ctypes.POINTER(VP), VP]),
    "precode_frame_symbols": (I, [VP, VP, VP, I, VP, VP]),
    "precode_frame_factors": (I, [VP, VP, VP, VP, VP]),
    "precode_frame_release": (I, [VP, VP]),
    "precode_batch": (I, [VP, ctypes.POINTER(Job), I, I, VP]),
    "precode_batch_plan_create": (I, [VP, ctypes.POINTER(Job), I, I, ctypes.POINTER(VP)]),
    "precode_batch_plan_launch": (I, [VP, VP]),
    "precode_batch_plan_launches": (I, [VP]),
    "precode_batch_plan_fused_jobs": (I, [VP]),
    "precode_autotune_reset": (None, []),
    "precode_batch_plan_destroy": (I, [VP]),
    "precode_serve": (I, [VP, ctypes.POINTER(ServeJob), I, ctypes.POINTER(ServeConfig),
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ServeStats)]),
}

_lib = None


class PrecodeError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().precode_strerror(code).decode()
        super().__init__("%s failed: %s (%d)" % (what or "precode call", msg, code))


def load() -> ctypes.CDLL:
    """Loads the in-tree libprecode.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libprecode.so is not built; run `python -m paper_1804_10987_amd.build` "
                              "(the HIP library is required: there is no fallback)")
        # torch ships its own HIP runtime: load it first, so that this library
        # binds to the same runtime as the tensors it is handed (whichever
        # libamdhip64 a process loads first serves both)
        import torch  # noqa: F401

        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int, what: str = "") -> None:
    if code != OK:
        raise PrecodeError(code, what)
