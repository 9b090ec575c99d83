"""ctypes declarations mirroring include/sft.h.  Loads the in-tree libsft.so
and fails loudly when it has not been built: there is no other path."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsft.so")

SFT_OK, SFT_E_INVALID, SFT_E_UNSUPPORTED, SFT_E_NOMEM, SFT_E_DEVICE, SFT_E_CAPACITY, SFT_E_NONFINITE = range(7)
SFT_C64, SFT_C128 = 1, 2
SFT_MODE_EXACT, SFT_MODE_GENERAL, SFT_MODE_ITERATIVE = 0, 1, 2
(SFT_FLAG_LEARNED, SFT_FLAG_SYNC, SFT_FLAG_CHECK_FINITE, SFT_FLAG_AUTOTUNE, SFT_FLAG_FFT64, SFT_FLAG_SP_ALL,
 SFT_FLAG_UNKNOWN_K) = 1, 2, 4, 8, 16, 32, 64
SFT_MAX_RSHIFTS = 64

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "sft_plan", "sft_exact", "sft_general", "sft_iterative", "sft_batch", "sft_syndromes", "sft_plan_get", "sft_destroy",
    "sft_status_str", "sft_last_error", "sft_abi_version",
    "sft_mlp_create", "sft_mlp_destroy", "sft_mlp_get_params", "sft_mlp_set_params", "sft_mlp_forward",
    "sft_mlp_grad", "sft_mlp_train_step", "sft_mlp_last_error", "sft_plan_attach_mlp", "sft_features",
    "sft_autotune", "sft_unknown_k", "sft_exact_noalloc",
]
MLP_FEATURES, MLP_CLASSES, MLP_PARAMS = 32, 5, 21381


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("m", ctypes.c_int64),
        ("l", ctypes.c_int32), ("r", ctypes.c_int32), ("in_dtype", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64),
        ("tau_zero", ctypes.c_double), ("tau_rank", ctypes.c_double), ("tau_res", ctypes.c_double),
        ("tau_amp", ctypes.c_double), ("c_res", ctypes.c_double), ("delta_grid", ctypes.c_double),
        ("delta_mag", ctypes.c_double), ("target_recovery", ctypes.c_double),
    ]


class SparseOut(ctypes.Structure):
    _fields_ = [
        ("loc_dev", ctypes.c_void_p), ("val_dev", ctypes.c_void_p),
        ("capacity", ctypes.c_int64), ("count_dev", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("active_bins", ctypes.c_int64), ("flagged_bins", ctypes.c_int64), ("cs_bins", ctypes.c_int64),
        ("mlp_fallbacks", ctypes.c_int64), ("entries", ctypes.c_int64), ("overflowed", ctypes.c_int64),
        ("nonfinite", ctypes.c_int64), ("stage_ms", ctypes.c_double * 4),
        ("gather_ms", ctypes.c_double * 2),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("stage_ms", "gather_ms")}
        d["stage_ms"] = list(self.stage_ms)
        d["gather_ms"] = list(self.gather_ms)
        return d


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("m", ctypes.c_int64), ("d", ctypes.c_int64),
        ("l", ctypes.c_int32), ("r", ctypes.c_int32), ("in_dtype", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("n_signals", ctypes.c_int32),
        ("rshifts", ctypes.c_int64 * SFT_MAX_RSHIFTS),
        ("tau_zero", ctypes.c_double), ("tau_rank", ctypes.c_double), ("tau_res", ctypes.c_double),
        ("tau_amp", ctypes.c_double), ("c_res", ctypes.c_double), ("delta_grid", ctypes.c_double),
        ("delta_mag", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
    ]


_lib = None


def load():
    """The loaded library (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the sFFT-DT path runs only through the HIP library)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.sft_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), i64, vp]
    lib.sft_plan.restype = st
    for name in ("sft_exact", "sft_general", "sft_iterative"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, ctypes.POINTER(SparseOut), ctypes.POINTER(Stats)]
        f.restype = st
    lib.sft_unknown_k.argtypes = [vp, vp, ctypes.POINTER(SparseOut), ctypes.POINTER(Stats), ctypes.POINTER(i64)]
    lib.sft_unknown_k.restype = st
    lib.sft_exact_noalloc.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(SparseOut), vp]
    lib.sft_exact_noalloc.restype = st
    lib.sft_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(SparseOut), ctypes.POINTER(Stats)]
    lib.sft_batch.restype = st
    lib.sft_syndromes.argtypes = [vp, vp, vp]
    lib.sft_syndromes.restype = st
    lib.sft_plan_get.argtypes = [vp, i64, ctypes.POINTER(PlanInfo)]
    lib.sft_plan_get.restype = st
    lib.sft_destroy.argtypes = [vp]
    lib.sft_destroy.restype = None
    lib.sft_status_str.argtypes = [st]
    lib.sft_status_str.restype = ctypes.c_char_p
    lib.sft_last_error.argtypes = []
    lib.sft_last_error.restype = ctypes.c_char_p
    lib.sft_abi_version.argtypes = []
    lib.sft_abi_version.restype = ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.sft_autotune.argtypes = [i64, i64, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(i64),
                                 ctypes.POINTER(ctypes.c_int32), dp, dp]
    lib.sft_autotune.restype = st
    fp = ctypes.POINTER(ctypes.c_float)
    lib.sft_mlp_create.argtypes = [ctypes.POINTER(vp), ctypes.c_uint64, vp]
    lib.sft_mlp_destroy.argtypes = [vp]
    lib.sft_mlp_destroy.restype = None
    lib.sft_mlp_get_params.argtypes = [vp, fp, i64]
    lib.sft_mlp_set_params.argtypes = [vp, fp, i64]
    lib.sft_mlp_forward.argtypes = [vp, vp, i64, vp]
    lib.sft_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.sft_mlp_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, vp]
    lib.sft_mlp_last_error.argtypes = []
    lib.sft_mlp_last_error.restype = ctypes.c_char_p
    lib.sft_plan_attach_mlp.argtypes = [vp, vp]
    lib.sft_features.argtypes = [vp, vp, vp, vp, i64, vp]
    for name in ("sft_mlp_create", "sft_mlp_get_params", "sft_mlp_set_params", "sft_mlp_forward", "sft_mlp_grad",
                 "sft_mlp_train_step", "sft_plan_attach_mlp", "sft_features"):
        getattr(lib, name).restype = st
    _lib = lib
    return lib


class SftError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def check(status: int, what: str = ""):
    if status != SFT_OK:
        lib = load()
        name = lib.sft_status_str(status).decode()
        detail = (lib.sft_mlp_last_error() if what.startswith("sft_mlp") else lib.sft_last_error()).decode()
        raise SftError(status, f"{what}: {name}: {detail}")
