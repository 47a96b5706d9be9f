"""ctypes binding of libsigkernel.so (argument marshalling only).

Every computation runs in the HIP kernels of ``csrc/``; this module only turns
torch tensors into the plain pointers and sizes of ``include/sigkernel.h``.
If the library has not been built the first call raises immediately: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsigkernel.so")

SK_OK = 0
SK_ERR_NULL = -1
SK_ERR_SHAPE = -2
SK_ERR_ORDER = -3
SK_ERR_WORKSPACE = -4
SK_ERR_FLAGS = -5
SK_ERR_HIP = -6
SK_ERR_UNSUPPORTED = -7
SK_ERR_STATE = -8
SK_ERR_VALUE = -9

SK_SYMMETRIC = 1 << 0
SK_NO_DIAG = 1 << 1
SK_MMD2_GRAD = 1 << 2
SK_GRAM_BF16 = 1 << 3
SK_GRAM_F16 = 1 << 4
SK_IMPLICIT = 1 << 5

SK_OP_PAIR = 0
SK_OP_GRAM = 1
SK_OP_GRAM_BACKWARD = 2
SK_OP_MMD2 = 3
SK_OP_CORRECTOR_FEATURES = 4
SK_OP_CORRECTOR_BACKWARD = 5
SK_OP_CORRECTOR_PREDICT = 6
SK_OP_PAIR_LIFTED = 7
SK_OP_GRAM_LIFTED = 8

SK_STATIC_LINEAR = 0
SK_STATIC_RBF = 1
SK_CHANNEL_STATS_WORKSPACE_BYTES = 32832

# Every symbol the header declares (checked by the CPU test suite).
EXPORTED = (
    "sigkernel_pair",
    "sigkernel_gram",
    "sigkernel_gram_noalloc",
    "sigkernel_gram_noalloc_max_bytes",
    "sigkernel_gram_backward",
    "sigkernel_mmd2",
    "sigkernel_increment_gram",
    "sigkernel_workspace_bytes",
    "sigkernel_status_string",
    "sigkernel_version",
    "sigkernel_tune_key",
    "sigkernel_tune_set",
    "sigkernel_tune_get",
    "sigkernel_tune_list",
    "sigkernel_tune_clear",
    "sigkernel_autotune",
    "sigkernel_graph_begin",
    "sigkernel_graph_end",
    "sigkernel_graph_launch",
    "sigkernel_graph_destroy",
    "sigkernel_corrector_param_count",
    "sigkernel_corrector_act_elems",
    "sigkernel_corrector_features",
    "sigkernel_corrector_forward",
    "sigkernel_corrector_backward",
    "sigkernel_corrector_loss",
    "sigkernel_adam_step",
    "sigkernel_channel_stats",
    "sigkernel_corrector_predict",
    "sigkernel_pair_lifted",
    "sigkernel_gram_lifted",
    "sigkernel_reduced_measure",
    "sigkernel_reduced_measure_support",
)


class SkPaths(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
        ("n_paths", ctypes.c_int64),
        ("len", ctypes.c_int32),
        ("dim", ctypes.c_int32),
    ]


class SkStaticKernel(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("sigma", ctypes.c_double),
    ]


class SkTuneKey(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("dyadic_order", ctypes.c_int32),
        ("symmetric", ctypes.c_int32),
        ("ragged", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("x_len", ctypes.c_int32),
        ("y_len", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class SkTune(ctypes.Structure):
    _fields_ = [
        ("run", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("pair_blocks_per_cu", ctypes.c_int32),
        ("pair_bands", ctypes.c_int32),
    ]


class SigKernelError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lib = None


def load():
    """Load libsigkernel.so; raise if it is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libsigkernel.so not found at {LIB_PATH}: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(SkPaths)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    i64 = ctypes.c_int64
    lib.sigkernel_pair.argtypes = [P, P, i32, u32, vp, vp, sz, vp]
    lib.sigkernel_pair.restype = i32
    lib.sigkernel_gram.argtypes = [P, P, i32, u32, vp, vp, sz, vp]
    lib.sigkernel_gram.restype = i32
    lib.sigkernel_gram_noalloc.argtypes = [P, P, i32, u32, vp, vp]
    lib.sigkernel_gram_noalloc.restype = i32
    lib.sigkernel_gram_noalloc_max_bytes.argtypes = []
    lib.sigkernel_gram_noalloc_max_bytes.restype = sz
    dbl = ctypes.c_double
    lib.sigkernel_reduced_measure.argtypes = [vp, vp, i32, dbl, dbl, i32, vp, vp, vp, vp]
    lib.sigkernel_reduced_measure.restype = i32
    lib.sigkernel_reduced_measure_support.argtypes = [vp, vp, i32, i32, i32, i32, dbl, vp, vp,
                                                      vp, vp]
    lib.sigkernel_reduced_measure_support.restype = i32
    SKp = ctypes.POINTER(SkStaticKernel)
    for name in ("sigkernel_pair_lifted", "sigkernel_gram_lifted"):
        getattr(lib, name).argtypes = [P, P, i32, u32, SKp, vp, vp, sz, vp]
        getattr(lib, name).restype = i32
    lib.sigkernel_gram_backward.argtypes = [P, P, i32, u32, vp, vp, vp, vp, sz, vp]
    lib.sigkernel_gram_backward.restype = i32
    lib.sigkernel_mmd2.argtypes = [P, P, i32, u32, vp, vp, vp, sz, vp]
    lib.sigkernel_mmd2.restype = i32
    lib.sigkernel_increment_gram.argtypes = [P, P, i32, u32, vp, i64, vp]
    lib.sigkernel_increment_gram.restype = i32
    lib.sigkernel_workspace_bytes.argtypes = [i32, P, P, i32, u32]
    lib.sigkernel_workspace_bytes.restype = sz
    lib.sigkernel_status_string.argtypes = [i32]
    lib.sigkernel_status_string.restype = ctypes.c_char_p
    lib.sigkernel_version.argtypes = []
    lib.sigkernel_version.restype = ctypes.c_char_p
    K, T = ctypes.POINTER(SkTuneKey), ctypes.POINTER(SkTune)
    lib.sigkernel_tune_key.argtypes = [i32, P, P, i32, u32, K]
    lib.sigkernel_tune_key.restype = i32
    lib.sigkernel_tune_set.argtypes = [K, T]
    lib.sigkernel_tune_set.restype = i32
    lib.sigkernel_tune_get.argtypes = [K, T]
    lib.sigkernel_tune_get.restype = i32
    lib.sigkernel_tune_list.argtypes = [K, T, ctypes.c_int64]
    lib.sigkernel_tune_list.restype = ctypes.c_int64
    lib.sigkernel_tune_clear.argtypes = []
    lib.sigkernel_tune_clear.restype = None
    lib.sigkernel_autotune.argtypes = [i32, P, P, i32, u32, vp, vp, sz, i32, vp, T,
                                       ctypes.POINTER(ctypes.c_float)]
    lib.sigkernel_autotune.restype = i32
    lib.sigkernel_graph_begin.argtypes = [vp]
    lib.sigkernel_graph_begin.restype = i32
    lib.sigkernel_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
    lib.sigkernel_graph_end.restype = i32
    lib.sigkernel_graph_launch.argtypes = [vp, vp]
    lib.sigkernel_graph_launch.restype = i32
    lib.sigkernel_graph_destroy.argtypes = [vp]
    lib.sigkernel_graph_destroy.restype = i32
    i64, f32 = ctypes.c_int64, ctypes.c_float
    lib.sigkernel_corrector_param_count.argtypes = []
    lib.sigkernel_corrector_param_count.restype = i64
    lib.sigkernel_corrector_act_elems.argtypes = []
    lib.sigkernel_corrector_act_elems.restype = i64
    lib.sigkernel_corrector_features.argtypes = [P, P, vp, vp, vp, vp, sz, vp]
    lib.sigkernel_corrector_features.restype = i32
    lib.sigkernel_corrector_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.sigkernel_corrector_forward.restype = i32
    lib.sigkernel_corrector_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, sz, vp]
    lib.sigkernel_corrector_backward.restype = i32
    lib.sigkernel_corrector_loss.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    lib.sigkernel_corrector_loss.restype = i32
    lib.sigkernel_adam_step.argtypes = [vp, vp, vp, vp, i64, vp, f32, f32, f32, f32, vp]
    lib.sigkernel_adam_step.restype = i32
    lib.sigkernel_channel_stats.argtypes = [vp, i32, vp, i64, i32, vp, vp, vp, sz, vp]
    lib.sigkernel_channel_stats.restype = i32
    lib.sigkernel_corrector_predict.argtypes = [P, P, i32, vp, vp, vp, f32, f32, vp, vp, vp, vp,
                                                sz, vp]
    lib.sigkernel_corrector_predict.restype = i32
    _lib = lib
    cache = os.environ.get("SIGKERNEL_TUNE_CACHE")
    if cache and os.path.exists(cache):
        from .tuning import load_cache
        load_cache(cache)
    return lib


def status_string(status: int) -> str:
    return load().sigkernel_status_string(int(status)).decode()


def version() -> str:
    return load().sigkernel_version().decode()


def check(status: int, what: str) -> None:
    if status != SK_OK:
        raise SigKernelError(status, what)
