"""ctypes declarations for librayshoot.so (the C ABI in include/rayshoot.h).

Argument marshalling only. Loading fails loudly if the library has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librayshoot.so")

RS_OK = 0
RS_EINVAL = -1
RS_ENOMEM = -2
RS_EHIP = -3
RS_EBUSY = -4
RS_ECANCELED = -5
RS_FP32 = 0
RS_MIXED = 1
RS_ACCUMULATE = 1
RS_EXACT_RECHECK = 2

_ERRNAMES = {RS_EINVAL: "RS_EINVAL", RS_ENOMEM: "RS_ENOMEM", RS_EHIP: "RS_EHIP",
             RS_EBUSY: "RS_EBUSY", RS_ECANCELED: "RS_ECANCELED"}


class RayshootError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {message}")
        self.code = code


class MapParams(ctypes.Structure):
    _fields_ = [("sigma_star", ctypes.c_double), ("sigma_c", ctypes.c_double), ("gamma", ctypes.c_double),
                ("sx0", ctypes.c_double), ("sy0", ctypes.c_double),
                ("sw", ctypes.c_double), ("sh", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("i0", ctypes.c_int64), ("i1", ctypes.c_int64),
                ("j0", ctypes.c_int64), ("j1", ctypes.c_int64),
                ("tx0", ctypes.c_double), ("ty0", ctypes.c_double),
                ("tw", ctypes.c_double), ("th", ctypes.c_double),
                ("npx", ctypes.c_int64), ("npy", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("flags", ctypes.c_int32)]


class MapStats(ctypes.Structure):
    _fields_ = [("rays_shot", ctypes.c_uint64), ("rays_in_map", ctypes.c_uint64),
                ("rays_out", ctypes.c_uint64), ("rays_singular", ctypes.c_uint64),
                ("rays_rechecked", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("n_shapes", ctypes.c_int32),
                ("rays_per_lane", (ctypes.c_int32 * 2) * 8), ("threads", ctypes.c_int32 * 8),
                ("ms", ctypes.c_double * 8), ("sample_interactions", ctypes.c_double)]


_lib = None

VP = ctypes.c_void_p
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
INT = ctypes.c_int


def _declare(lib):
    P = ctypes.POINTER
    sigs = {
        "rs_version": ([], ctypes.c_char_p),
        "rs_last_error": ([], ctypes.c_char_p),
        "rs_workspace_bytes": ([P(MapParams), I64], SZ),
        "rs_make_map": ([P(MapParams), VP, VP, I64, VP, VP, SZ, VP], INT),
        "rs_ray_pixels": ([P(MapParams), VP, VP, I64, VP, VP, SZ, VP], INT),
        "rs_read_stats": ([VP, P(MapStats), VP], INT),
        "rs_profile_enable": ([INT], INT),
        "rs_profile_read": ([P(ctypes.c_double), P(I64), P(ctypes.c_double)], INT),
        "rs_tune": ([P(MapParams), VP, VP, I64, VP, VP, SZ, I64, VP, P(TuneResult)], INT),
        "rs_set_shape": ([INT, ctypes.POINTER(INT)], INT),
        "rs_tune_save": ([ctypes.c_char_p], INT),
        "rs_tune_load": ([ctypes.c_char_p], INT),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def check(rc: int) -> None:
    if rc != RS_OK:
        msg = lib().rs_last_error().decode(errors="replace")
        raise RayshootError(rc, msg)


def exported_symbols():
    """Names of the C-ABI functions this binding declares."""
    return ["rs_version", "rs_last_error", "rs_workspace_bytes", "rs_make_map", "rs_ray_pixels",
            "rs_read_stats", "rs_profile_enable", "rs_profile_read", "rs_tune", "rs_set_shape",
            "rs_tune_save", "rs_tune_load"]
