"""ctypes binding of ``libexpm.so`` (the C ABI declared in include/expm.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.  The
library must have been built (``paper_1710_10989_amd.build.build()``); importing this module
without it raises, there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexpm.so")

EXPM_OK, EXPM_E_INVALID_ARG, EXPM_E_NONFINITE, EXPM_E_WORKSPACE, EXPM_E_HIP, EXPM_E_UNSUPPORTED = range(6)
EXPM_F64, EXPM_C128 = 0, 1
EXPM_PREC_FP64, EXPM_PREC_FP32, EXPM_PREC_BF16X3, EXPM_PREC_FP32_ALL = 0, 1, 2, 3
EXPM_SEL_PLAIN, EXPM_SEL_ALPHA, EXPM_SEL_LEARNED = 0, 1, 2
EXPM_FLAG_PS, EXPM_FLAG_PADE, EXPM_FLAG_TRI = 1, 2, 4

EXPORTED = ("expm_status_string", "expm_theta", "expm_select_rule", "expm_workspace_bytes",
            "expm_select", "expm_taylor", "expm_batched", "expm_batched_noalloc", "expm_batched_stage", "expm_batched_uniform",
            "expm_magnus4_step", "expm_tune_set", "expm_tune_get", "expm_tune_limits", "expm_features", "expm_mlp_scratch_bytes", "expm_mlp_param_count", "expm_mlp_forward",
            "expm_mlp_grad", "expm_mlp_adam", "expm_learned_set", "expm_learned_counts")


class ExpmOpts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("prec", ctypes.c_int32), ("sel", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("u", ctypes.c_double)]


class ExpmTune(ctypes.Structure):
    _fields_ = [("arrangement", ctypes.c_int32 * 3), ("small_kernel", ctypes.c_int32),
                ("per_cu", ctypes.c_int32 * 6), ("tiles_per_launch", ctypes.c_int32 * 4)]


class ExpmError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (status %d)" % (what, status_string(code), code))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libexpm.so is not built; run paper_1710_10989_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, dbl, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
        op = ctypes.POINTER(ExpmOpts)
        L.expm_status_string.argtypes = [i32]; L.expm_status_string.restype = ctypes.c_char_p
        L.expm_theta.argtypes = [i32, dbl, ctypes.POINTER(dbl)]; L.expm_theta.restype = i32
        L.expm_select_rule.argtypes = [ctypes.POINTER(dbl), i32, dbl, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.expm_select_rule.restype = i32
        L.expm_workspace_bytes.argtypes = [i64, i64, op]; L.expm_workspace_bytes.restype = sz
        L.expm_select.argtypes = [vp, i64, op, vp, vp, vp, sz, vp]; L.expm_select.restype = i32
        L.expm_taylor.argtypes = [vp, vp, i64, op, vp, vp, vp, vp, sz, vp]; L.expm_taylor.restype = i32
        L.expm_batched.argtypes = [vp, vp, vp, vp, i64, i64, op, vp, vp, vp, vp, sz, vp]
        L.expm_batched.restype = i32
        L.expm_batched_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, op, vp, vp, vp, vp]
        L.expm_batched_noalloc.restype = i32
        L.expm_batched_stage.argtypes = [vp, vp, vp, vp, i64, i64, op, vp, vp, vp, vp, sz, vp, i32]
        L.expm_batched_stage.restype = i32
        L.expm_batched_uniform.argtypes = [vp, vp, i64, i64, op, vp, vp, vp, vp, sz, vp]
        L.expm_batched_uniform.restype = i32
        L.expm_magnus4_step.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, i64, dbl, op, vp, vp, vp, vp]
        L.expm_magnus4_step.restype = i32
        tp = ctypes.POINTER(ExpmTune)
        L.expm_tune_set.argtypes = [tp]; L.expm_tune_set.restype = i32
        L.expm_tune_get.argtypes = [tp]; L.expm_tune_get.restype = i32
        L.expm_tune_limits.argtypes = [tp]; L.expm_tune_limits.restype = i32
        L.expm_features.argtypes = [vp, vp, vp, i64, i64, op, vp, vp, vp, vp, sz, vp]
        L.expm_features.restype = i32
        L.expm_mlp_scratch_bytes.argtypes = [i32]; L.expm_mlp_scratch_bytes.restype = sz
        L.expm_mlp_param_count.argtypes = []; L.expm_mlp_param_count.restype = i32
        L.expm_mlp_forward.argtypes = [vp, vp, i32, vp, vp, sz, vp]; L.expm_mlp_forward.restype = i32
        L.expm_mlp_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp, sz, vp]; L.expm_mlp_grad.restype = i32
        L.expm_mlp_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]; L.expm_mlp_adam.restype = i32
        L.expm_learned_set.argtypes = [vp, vp, vp]; L.expm_learned_set.restype = i32
        L.expm_learned_counts.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.expm_learned_counts.restype = i32
        _lib = L
    return _lib


def status_string(code):
    return lib().expm_status_string(int(code)).decode()


def check(code, what):
    if code != EXPM_OK:
        raise ExpmError(code, what)
