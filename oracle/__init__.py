"""Python loader for the FP64 CPU oracle (test infrastructure only).

Only tests, the smoke check and the bench's CPU-baseline leg import this
package. It compiles ``oracle.c`` with gcc (-O2, no fast-math, no FP
contraction) into ``liboracle.so`` next to this file and calls it via ctypes.
It shares nothing with the HIP product path: the parameter struct below is
this package's own definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-pthread"]

RAY_OUT = -1
RAY_SINGULAR = -2


class OracleParams(ctypes.Structure):
    _fields_ = [("sigma_c", ctypes.c_double), ("gamma", ctypes.c_double),
                ("sx0", ctypes.c_double), ("sy0", ctypes.c_double),
                ("sw", ctypes.c_double), ("sh", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("i0", ctypes.c_int64), ("i1", ctypes.c_int64),
                ("j0", ctypes.c_int64), ("j1", ctypes.c_int64),
                ("tx0", ctypes.c_double), ("ty0", ctypes.c_double),
                ("tw", ctypes.c_double), ("th", ctypes.c_double),
                ("npx", ctypes.c_int64), ("npy", ctypes.c_int64),
                ("random_rays", ctypes.c_int64), ("seed", ctypes.c_uint64)]


def build(force: bool = True, extra_flags=(), src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (always when force, else only if the output is missing)."""
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Lib:
    """A loaded oracle library (the default one, or a test build at another path)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_make_map.argtypes = [P(OracleParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_make_map.restype = ctypes.c_int
        lib.oracle_ray_pixels.argtypes = [P(OracleParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_ray_pixels.restype = ctypes.c_int
        lib.oracle_philox4x64.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_philox4x64.restype = None
        self.lib = lib
        self.path = path

    def make_map(self, params, lens_xy, lens_m=None, near_tol=1e-9, near_cap=4096, nthreads=None):
        return make_map(params, lens_xy, lens_m, near_tol, near_cap, nthreads, _use=self.lib)

    def ray_pixels(self, params, lens_xy, lens_m=None, nthreads=None):
        return ray_pixels(params, lens_xy, lens_m, nthreads, _use=self.lib)

    def philox4x64(self, counter, key):
        return philox4x64(counter, key, _use=self.lib)


_default = None


def _load():
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build(force=False)
        _default = _Lib(LIB)
    return _default.lib


def load(path: str) -> _Lib:
    """Load an oracle library built at ``path`` (used by the pin-sensitivity tests)."""
    return _Lib(path)


def default() -> _Lib:
    _load()
    return _default


def _params(p: dict) -> OracleParams:
    """Missing random_rays / seed mean the regular grid."""
    return OracleParams(*(p.get(k, 0) if k in ("random_rays", "seed") else p[k] for k, _ in OracleParams._fields_))


def _lens(lens_xy, lens_m):
    xy = np.ascontiguousarray(np.asarray(lens_xy, dtype=np.float64).reshape(-1, 2))
    m = None if lens_m is None else np.ascontiguousarray(np.asarray(lens_m, dtype=np.float64).reshape(-1))
    if m is not None and m.shape[0] != xy.shape[0]:
        raise ValueError("lens_m length differs from lens_xy")
    return xy, m


def default_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 64))


def make_map(params: dict, lens_xy, lens_m=None, near_tol: float = 1e-9, near_cap: int = 4096,
             nthreads: Optional[int] = None, _use=None):
    """Return (map uint32 [npy, npx], stats dict) for the params' ray window."""
    lib = _use or _load()
    xy, m = _lens(lens_xy, lens_m)
    p = _params(params)
    out = np.zeros((int(params["npy"]), int(params["npx"])), dtype=np.uint32)
    counts = np.zeros(4, dtype=np.uint64)
    near = np.zeros((max(near_cap, 1), 2), dtype=np.int64)
    rc = lib.oracle_make_map(ctypes.byref(p), xy.ctypes.data if xy.shape[0] else None,
                             None if m is None else m.ctypes.data, xy.shape[0],
                             out.ctypes.data, counts.ctypes.data, float(near_tol),
                             near.ctypes.data, near_cap, nthreads or default_threads())
    if rc != 0:
        raise RuntimeError(f"oracle_make_map failed ({rc})")
    n_near = int(counts[3])
    stats = dict(rays_in_map=int(counts[0]), rays_out=int(counts[1]), rays_singular=int(counts[2]),
                 near_edge=n_near, near_edge_rays=[tuple(r) for r in near[:min(n_near, near_cap)]])
    return out, stats


def philox4x64(counter, key, _use=None):
    """Philox4x64-10 block (four uint64) of counter (4 words) under key (2 words)."""
    lib = _use or _load()
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(2))
    out = np.zeros(4, dtype=np.uint64)
    lib.oracle_philox4x64(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def ray_pixels(params: dict, lens_xy, lens_m=None, nthreads: Optional[int] = None, _use=None):
    """Per-ray (pix, u, v) over the window, row-major: pix = v*npx+u, -1 out, -2 singular."""
    lib = _use or _load()
    xy, m = _lens(lens_xy, lens_m)
    p = _params(params)
    n = int((params["i1"] - params["i0"]) * (params["j1"] - params["j0"]))
    pix = np.empty(n, dtype=np.int64)
    u = np.empty(n, dtype=np.float64)
    v = np.empty(n, dtype=np.float64)
    rc = lib.oracle_ray_pixels(ctypes.byref(p), xy.ctypes.data if xy.shape[0] else None,
                               None if m is None else m.ctypes.data, xy.shape[0],
                               pix.ctypes.data, u.ctypes.data, v.ctypes.data,
                               nthreads or default_threads())
    if rc != 0:
        raise RuntimeError(f"oracle_ray_pixels failed ({rc})")
    return pix, u, v
