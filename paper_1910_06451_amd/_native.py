"""ctypes binding of libfastron_fk.so (the C ABI declared in include/fastron_fk.h).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch supplies device memory and the current stream. The library
must have been built (``python -m paper_1910_06451_amd.build``); there is no
fallback path -- a missing library raises ``FastronLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastron_fk.so")

FASTRON_OK = 0
FASTRON_NOT_CONVERGED = 1
FASTRON_EINVAL = -1
FASTRON_EUNSUPPORTED = -2
FASTRON_EHIP = -3
FASTRON_ENOMEM = -4
FASTRON_EDEVICE = -5

SCORE_FP32 = 0x0
SCORE_BF16 = 0x1
SCORE_VALU = 0x2
BF16_PLAIN = 0x00
BF16_SPLIT2 = 0x10
BF16_SPLIT3 = 0x20

EXPORTED = [
    "fastron_control_point_frames", "fastron_fk_points", "fastron_model_bytes", "fastron_support_prep", "fastron_fk_score_prepared",
    "fastron_score_rational", "fastron_fk_score", "fastron_gram_update", "fastron_gram_update_points", "fastron_train", "fastron_train_f64",
    "fastron_train_points", "fastron_train_points_f64", "fastron_train_batch", "fastron_label_capsule_box",
    "fastron_tune_set", "fastron_tune_get", "fastron_last_error", "fastron_version", "fastron_batch_create",
    "fastron_batch_prepare", "fastron_batch_score", "fastron_batch_autotune", "fastron_batch_capture",
    "fastron_batch_replay", "fastron_batch_tile_queries", "fastron_batch_destroy", "fastron_mlp_create",
    "fastron_mlp_destroy", "fastron_mlp_param_count", "fastron_mlp_set_params", "fastron_mlp_get_params",
    "fastron_mlp_fit_standardisation", "fastron_mlp_forward", "fastron_mlp_gradients", "fastron_mlp_train_epoch",
    "fastron_mlp_screen", "fastron_mlp_screen_workspace_bytes", "fastron_rbf_score", "fastron_rbf_train",
    "fastron_rbf_train_f64", "fastron_active_samples", "fastron_fk_score_noalloc", "fastron_mlp_get_adam_state",
    "fastron_active_relabel", "fastron_batch_get_shape", "fastron_batch_set_shape",
]


class FastronLibraryMissing(RuntimeError):
    pass


class FastronError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fastron status {status}: {msg}")
        self.status = status


class Chain(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.POINTER(ctypes.c_double)), ("d", ctypes.POINTER(ctypes.c_double)),
                ("theta", ctypes.POINTER(ctypes.c_double)), ("type", ctypes.POINTER(ctypes.c_int32)),
                ("base", ctypes.POINTER(ctypes.c_double))]


class CPoints(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("frame", ctypes.POINTER(ctypes.c_int32)),
                ("offset", ctypes.POINTER(ctypes.c_double))]


class Model(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int64), ("M", ctypes.c_int32), ("gamma", ctypes.c_float),
                ("data", ctypes.c_void_p), ("bytes", ctypes.c_int64)]


_lib = None


def lib():
    """Load the HIP library (once). Raises FastronLibraryMissing if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FastronLibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -m paper_1910_06451_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
    ch, cp, md = ctypes.POINTER(Chain), ctypes.POINTER(CPoints), ctypes.POINTER(Model)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "fastron_control_point_frames": ([ch, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                                         i32),
        "fastron_fk_points": ([ch, cp, vp, i64, vp, vp], i32),
        "fastron_model_bytes": ([i64, i32], i64),
        "fastron_support_prep": ([ch, cp, vp, vp, i64, f32, md, vp], i32),
        "fastron_fk_score_prepared": ([ch, cp, md, vp, i64, vp, vp, ctypes.c_uint32, vp], i32),
        "fastron_score_rational": ([ch, cp, f32, ctypes.c_uint32], i32),
        "fastron_fk_score": ([ch, cp, vp, vp, i64, f32, vp, i64, vp, vp, ctypes.c_uint32, vp], i32),
        "fastron_fk_score_noalloc": ([ch, cp, vp, vp, i64, f32, vp, i64, vp, vp, ctypes.c_uint32, vp], i32),
        "fastron_gram_update": ([ch, cp, vp, i64, f32, i64, f32, vp, vp, vp], i32),
        "fastron_gram_update_points": ([vp, i64, i32, f32, i64, f32, vp, vp, vp], i32),
        "fastron_train": ([ch, cp, vp, vp, i64, f32, f32, i64, i64, vp, vp, vp, pi64, pi64, vp, vp, i64, vp], i32),
        "fastron_train_f64": ([ch, cp, vp, vp, i64, f64, f64, i64, i64, vp, vp, vp, pi64, pi64, vp, vp, i64, vp],
                              i32),
        "fastron_train_points": ([vp, vp, i64, i32, f32, f32, i64, i64, vp, vp, vp, pi64, pi64, vp, vp, i64, vp],
                                 i32),
        "fastron_train_points_f64": ([vp, vp, i64, i32, f64, f64, i64, i64, vp, vp, vp, pi64, pi64, vp, vp, i64,
                                      vp], i32),
        "fastron_train_batch": ([vp, vp, i32, pi64, i32, f32, f32, i64, i64, vp, vp, vp, pi64, pi64, vp], i32),
        "fastron_label_capsule_box": ([ch, vp, i64, f64, vp, i32, vp, vp, vp], i32),
        "fastron_batch_create": ([ch, cp, i32, pi64, pi64, f32, ctypes.POINTER(vp)], i32),
        "fastron_batch_prepare": ([vp, vp, vp, vp], i32),
        "fastron_batch_score": ([vp, vp, vp, vp, vp], i32),
        "fastron_batch_autotune": ([vp, vp, vp, vp, vp], i32),
        "fastron_batch_capture": ([vp, vp, vp, vp, vp], i32),
        "fastron_batch_replay": ([vp, vp], i32),
        "fastron_batch_tile_queries": ([vp], i32),
        "fastron_batch_get_shape": ([vp, pi32, pi32, pi32, pi32, pi32], i32),
        "fastron_batch_set_shape": ([vp, i32, i32, i32, i32, vp], i32),
        "fastron_batch_destroy": ([vp], None),
        "fastron_mlp_create": ([i32, i32, i64, ctypes.POINTER(vp)], i32),
        "fastron_mlp_destroy": ([vp], None),
        "fastron_mlp_param_count": ([vp], i64),
        "fastron_mlp_set_params": ([vp, vp, vp, vp, vp], i32),
        "fastron_mlp_get_params": ([vp, vp, vp, vp, vp, vp], i32),
        "fastron_mlp_get_adam_state": ([vp, vp, vp, pi64, vp], i32),
        "fastron_mlp_fit_standardisation": ([vp, vp, i64, vp], i32),
        "fastron_mlp_forward": ([vp, vp, i64, vp, vp], i32),
        "fastron_mlp_gradients": ([vp, vp, vp, i64, ctypes.POINTER(ctypes.c_float), vp], i32),
        "fastron_mlp_train_epoch": ([vp, vp, vp, vp, i64, i64, f32, ctypes.POINTER(ctypes.c_float), vp], i32),
        "fastron_mlp_screen": ([vp, ch, cp, md, vp, i64, f32, vp, vp, vp, pi64, vp, i64, vp], i32),
        "fastron_mlp_screen_workspace_bytes": ([i64, i32], i64),
        "fastron_rbf_score": ([vp, vp, i64, i32, f32, vp, i64, vp, vp, vp], i32),
        "fastron_rbf_train": ([vp, vp, i64, i32, f32, f32, i64, i64, vp, vp, vp, pi64, pi64, vp], i32),
        "fastron_rbf_train_f64": ([vp, vp, i64, i32, f64, f64, i64, i64, vp, vp, vp, pi64, pi64, vp, vp, i64, vp],
                                  i32),
        "fastron_active_samples": ([vp, vp, i64, i32, vp, i32, vp, i64, vp, vp, vp], i32),
        "fastron_active_relabel": ([vp, i64, vp, vp], i32),
        "fastron_tune_set": ([ctypes.c_char_p, i64], i32),
        "fastron_tune_get": ([ctypes.c_char_p], i64),
        "fastron_last_error": ([], ctypes.c_char_p),
        "fastron_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def tune_set(key: str, value: int) -> None:
    check(lib().fastron_tune_set(key.encode(), int(value)))


def tune_get(key: str) -> int:
    return int(lib().fastron_tune_get(key.encode()))


def last_error() -> str:
    return lib().fastron_last_error().decode()


def check(status: int, allow=(FASTRON_OK,)) -> int:
    if status not in allow:
        raise FastronError(status, last_error())
    return status


# --------------------------------------------------------------------------- #
# Host structs
# --------------------------------------------------------------------------- #
class HostChain:
    """Keeps the NumPy arrays behind a Chain / CPoints pair alive."""

    def __init__(self, arm):
        self.a = np.ascontiguousarray(arm.a, dtype=np.float64)
        n = self.a.shape[0]
        self.alpha = np.ascontiguousarray(arm.alpha, dtype=np.float64)
        self.d = np.ascontiguousarray(arm.d, dtype=np.float64)
        self.theta = np.ascontiguousarray(getattr(arm, "theta", np.zeros(n)), dtype=np.float64)
        self.type = np.ascontiguousarray(getattr(arm, "joint_type", np.zeros(n)), dtype=np.int32)
        base = getattr(arm, "base", None)
        self.base = None if base is None else np.ascontiguousarray(base, dtype=np.float64).reshape(16)
        self.frame = np.ascontiguousarray(arm.frames, dtype=np.int32)
        off = getattr(arm, "offsets", None)
        self.offset = None if off is None else np.ascontiguousarray(off, dtype=np.float64).reshape(-1)
        dp = lambda x: None if x is None else x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.chain = Chain(n, dp(self.a), dp(self.alpha), dp(self.d), dp(self.theta),
                           self.type.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dp(self.base))
        self.cpoints = CPoints(int(self.frame.shape[0]), self.frame.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               dp(self.offset))
        self.n = n
        self.M = int(self.frame.shape[0])
