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
RS_FARFIELD = 2
RS_ACCUMULATE = 1
RS_EXACT_RECHECK = 2
RS_RANDOM_RAYS = 4
RS_NOALLOC_SCRATCH_BYTES = 64 << 20

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
                ("mode", ctypes.c_int32), ("flags", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class MapStats(ctypes.Structure):
    _fields_ = [("rays_shot", ctypes.c_uint64), ("rays_in_map", ctypes.c_uint64),
                ("rays_out", ctypes.c_uint64), ("rays_singular", ctypes.c_uint64),
                ("rays_rechecked", ctypes.c_uint64), ("rays_rechecked_direct", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class MapRequest(ctypes.Structure):
    _fields_ = [("params", MapParams), ("lens_xy", ctypes.c_void_p), ("lens_m", ctypes.c_void_p),
                ("n_lens", ctypes.c_int64), ("map", ctypes.c_void_p)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("slice_ms", ctypes.c_double), ("starve_s", ctypes.c_double),
                ("max_waiting", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("completed", "canceled", "failed", "steps", "waiting", "active",
                                               "max_waiting", "hbm_in_use_bytes", "hbm_peak_bytes")] + \
               [(n, ctypes.c_double) for n in ("interactions", "gpu_busy_s", "maps_per_s", "latency_p50_s",
                                               "latency_p99_s", "latency_mean_s", "latency_max_s")] + \
               [("rejected_busy", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: (int(v) if isinstance(v, int) else float(v)) for k, v in
                ((k, getattr(self, k)) for k, _ in self._fields_)}


class TuneResult(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("n_shapes", ctypes.c_int32),
                ("rays_per_lane", (ctypes.c_int32 * 2) * 8), ("threads", ctypes.c_int32 * 8),
                ("ms", ctypes.c_double * 8), ("sample_interactions", ctypes.c_double)]


class TuneBatchResult(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int32), ("n", ctypes.c_int32), ("shape", ctypes.c_int32 * 16),
                ("blocks_per_cu", ctypes.c_int32 * 16), ("ms", ctypes.c_double * 16),
                ("sample_interactions", ctypes.c_double)]


class CompareResult(ctypes.Structure):
    _fields_ = [("rms_dm", ctypes.c_double), ("ks_d", ctypes.c_double), ("ks_p", ctypes.c_double),
                ("mean_mu_a", ctypes.c_double), ("mean_mu_b", ctypes.c_double),
                ("n_pix", ctypes.c_int64), ("n_both", ctypes.c_int64),
                ("n_zero_a", ctypes.c_int64), ("n_zero_b", ctypes.c_int64),
                ("max_a", ctypes.c_uint32), ("max_b", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


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
        "rs_make_map_noalloc": ([P(MapParams), VP, VP, I64, VP, P(MapStats), VP], INT),
        "rs_profile_enable": ([INT], INT),
        "rs_profile_read": ([P(ctypes.c_double), P(I64), P(ctypes.c_double)], INT),
        "rs_tune": ([P(MapParams), VP, VP, I64, VP, VP, SZ, I64, VP, P(TuneResult)], INT),
        "rs_set_shape": ([INT, ctypes.POINTER(INT)], INT),
        "rs_tune_save": ([ctypes.c_char_p], INT),
        "rs_tune_load": ([ctypes.c_char_p], INT),
        "rs_batch_workspace_bytes": ([P(MapRequest), ctypes.c_int32], SZ),
        "rs_make_maps": ([P(MapRequest), ctypes.c_int32, VP, SZ, VP], INT),
        "rs_batch_read_stats": ([VP, ctypes.c_int32, P(MapStats), VP], INT),
        "rs_tune_batch": ([P(MapRequest), ctypes.c_int32, VP, SZ, I64, VP, P(TuneBatchResult)], INT),
        "rs_server_create": ([P(ServerCfg), P(VP)], INT),
        "rs_server_submit": ([VP, P(MapParams), VP, VP, I64, VP, P(ctypes.c_uint64)], INT),
        "rs_server_poll": ([VP, ctypes.c_uint64, P(INT)], INT),
        "rs_server_wait": ([VP, ctypes.c_uint64, P(MapStats), P(ctypes.c_double)], INT),
        "rs_server_cancel": ([VP, ctypes.c_uint64], INT),
        "rs_server_get_stats": ([VP, P(ServerStats)], INT),
        "rs_server_destroy": ([VP], None),
        "rs_rays_per_pixel": ([P(MapParams)], ctypes.c_double),
        "rs_map_max": ([VP, I64, VP, VP], INT),
        "rs_map_histogram": ([VP, I64, ctypes.c_uint32, VP, VP], INT),
        "rs_delta_m": ([VP, I64, ctypes.c_double, VP, VP], INT),
        "rs_compare_workspace_bytes": ([ctypes.c_uint32, ctypes.c_uint32], SZ),
        "rs_compare_maps": ([VP, VP, I64, ctypes.c_double, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                             VP, SZ, P(CompareResult), VP], INT),
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
            "rs_read_stats", "rs_make_map_noalloc", "rs_profile_enable", "rs_profile_read", "rs_tune", "rs_set_shape",
            "rs_tune_save", "rs_tune_load", "rs_batch_workspace_bytes", "rs_make_maps",
            "rs_batch_read_stats", "rs_tune_batch", "rs_server_create", "rs_server_submit", "rs_server_poll", "rs_server_wait",
            "rs_server_cancel", "rs_server_get_stats", "rs_server_destroy", "rs_rays_per_pixel", "rs_map_max",
            "rs_map_histogram", "rs_delta_m", "rs_compare_workspace_bytes", "rs_compare_maps"]
