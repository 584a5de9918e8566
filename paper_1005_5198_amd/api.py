"""Python entry points over the C ABI: make_map, ray_pixels, read_stats.

PyTorch supplies device memory and the stream; every step of the computation
runs in the library's HIP kernels. Inputs given as numpy arrays are copied to
the device first.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L

MODES = {"fp32": L.RS_FP32, "mixed": L.RS_MIXED, "farfield": L.RS_FARFIELD}
SHAPES = {0: (4, 2), 1: (4, 4), 2: (8, 2), 3: (8, 4)}   # rays per lane (x, y) of each thread shape


def to_params(p: dict, mode: str = "mixed", accumulate: bool = False, exact_recheck: bool = False) -> L.MapParams:
    """Build the C parameter struct from a workloads-style dict (keys of MapParams).

    Optional keys: ``random_rays`` (true: Philox-random ray positions) and ``seed``."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    s = L.MapParams()
    for name, _ in L.MapParams._fields_:
        if name == "mode":
            s.mode = MODES[mode]
        elif name == "flags":
            s.flags = ((L.RS_ACCUMULATE if accumulate else 0) | (L.RS_EXACT_RECHECK if exact_recheck else 0) |
                       (L.RS_RANDOM_RAYS if p.get("random_rays") else 0))
        elif name == "seed":
            s.seed = int(p.get("seed", 0))
        else:
            setattr(s, name, p[name])
    return s


def _device():
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def lens_tensors(lens_xy, lens_m=None, device=None):
    """float64 device tensors [N,2] and [N] (or None) from numpy arrays or tensors."""
    device = device or _device()
    xy = torch.as_tensor(lens_xy, dtype=torch.float64).reshape(-1, 2).to(device).contiguous()
    m = None
    if lens_m is not None:
        m = torch.as_tensor(lens_m, dtype=torch.float64).reshape(-1).to(device).contiguous()
        if m.shape[0] != xy.shape[0]:
            raise ValueError("lens_m and lens_xy differ in length")
    return xy, m


def _ptr(t) -> Optional[int]:
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _hold(stream, *tensors) -> None:
    """Tensors made on the current stream but used by the library on another stream:
    tell the caching allocator, so that their memory is not handed out again before
    that stream's work on them has finished."""
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def workspace_bytes(params: dict, n_lens: int, mode: str = "mixed") -> int:
    c = to_params(params, mode)
    n = L.lib().rs_workspace_bytes(ctypes.byref(c), int(n_lens))
    if n == 0:
        L.check(L.RS_EINVAL)
    return int(n)


def new_workspace(params: dict, n_lens: int, mode: str = "mixed", device=None) -> torch.Tensor:
    return torch.empty(workspace_bytes(params, n_lens, mode), dtype=torch.uint8, device=device or _device())


def map_params(sigma_star: float, sigma_c: float, gamma: float, shoot, src, window=None) -> dict:
    """The parameter dict of one map: the macro model (Section 2, Eq. (sigma)), the shooting grid
    shoot = (x0, y0, w, h, nx, ny) of cell-centred rays, the source grid src = (x0, y0, w, h,
    npx, npy), and the ray window (i0, i1, j0, j1), the whole grid by default."""
    sx0, sy0, sw, sh, nx, ny = shoot
    tx0, ty0, tw, th, npx, npy = src
    i0, i1, j0, j1 = (0, int(nx), 0, int(ny)) if window is None else (int(v) for v in window)
    return dict(sigma_star=float(sigma_star), sigma_c=float(sigma_c), gamma=float(gamma),
                sx0=float(sx0), sy0=float(sy0), sw=float(sw), sh=float(sh), nx=int(nx), ny=int(ny),
                i0=i0, i1=i1, j0=j0, j1=j1,
                tx0=float(tx0), ty0=float(ty0), tw=float(tw), th=float(th), npx=int(npx), npy=int(npy))


def shoot_map(lens_xy, masses, sigma_star: float, sigma_c: float, gamma: float, shoot, src,
              mode: str = "mixed", **kwargs):
    """make_map with the model and grids given directly: lens positions [N, 2] and masses [N]
    (None for unit masses), sigma_star, sigma_c, gamma, shoot = (x0, y0, w, h, nx, ny) and
    src = (x0, y0, w, h, npx, npy). Returns the uint32 [npy, npx] count map; keyword
    arguments go to make_map."""
    return make_map(map_params(sigma_star, sigma_c, gamma, shoot, src), lens_xy, masses, mode=mode, **kwargs)


def make_map(params: dict, lens_xy, lens_m=None, mode: str = "mixed", out: Optional[torch.Tensor] = None,
             workspace: Optional[torch.Tensor] = None, accumulate: bool = False, stream=None,
             return_stats: bool = False, exact_recheck: bool = False):
    """Count map uint32 [npy, npx] of the params' ray window (Section 2, Eq. (sigma), Eq. (mu_ij)).

    Asynchronous on the stream unless return_stats is set (then it synchronises
    and also returns the counters as a dict).
    """
    dev = _device()
    xy, m = lens_tensors(lens_xy, lens_m, dev)
    c = to_params(params, mode, accumulate, exact_recheck)
    if out is None:
        out = torch.empty((int(params["npy"]), int(params["npx"])), dtype=torch.uint32, device=dev)
    if out.dtype != torch.uint32 or not out.is_contiguous() or tuple(out.shape) != (c.npy, c.npx):
        raise ValueError("out must be a contiguous uint32 tensor of shape (npy, npx)")
    if workspace is None:
        workspace = new_workspace(params, xy.shape[0], mode, dev)
    h = _stream_handle(stream)
    L.check(L.lib().rs_make_map(ctypes.byref(c), _ptr(xy), _ptr(m), xy.shape[0], out.data_ptr(),
                                workspace.data_ptr(), workspace.numel(), h))
    _hold(stream, xy, m, out, workspace)
    if return_stats:
        return out, read_stats(workspace, stream)
    return out


def make_map_noalloc(params: dict, lens_xy, lens_m=None, mode: str = "mixed", out: Optional[torch.Tensor] = None,
                     accumulate: bool = False, stream=None, return_stats: bool = False,
                     exact_recheck: bool = False):
    """make_map through the entry point that allocates nothing on the device: the library
    uses its static per-device scratch instead of a workspace. Calls that overlap on one
    device race (they share that scratch). With return_stats it synchronises and also
    returns the counters. Pass device tensors for the lenses and ``out`` to keep the
    binding itself from allocating."""
    dev = _device()
    xy, m = lens_tensors(lens_xy, lens_m, dev)
    c = to_params(params, mode, accumulate, exact_recheck)
    if out is None:
        out = torch.empty((int(params["npy"]), int(params["npx"])), dtype=torch.uint32, device=dev)
    if out.dtype != torch.uint32 or not out.is_contiguous() or tuple(out.shape) != (c.npy, c.npx):
        raise ValueError("out must be a contiguous uint32 tensor of shape (npy, npx)")
    st = L.MapStats() if return_stats else None
    L.check(L.lib().rs_make_map_noalloc(ctypes.byref(c), _ptr(xy), _ptr(m), xy.shape[0], out.data_ptr(),
                                        ctypes.byref(st) if st is not None else None, _stream_handle(stream)))
    _hold(stream, xy, m, out)
    if return_stats:
        return out, st.as_dict()
    return out


def ray_pixels(params: dict, lens_xy, lens_m=None, mode: str = "mixed", workspace=None, stream=None,
               return_stats: bool = False, exact_recheck: bool = False):
    """Per-ray pixel index int32 over the window (row-major): v*npx+u, -1 out, -2 singular."""
    dev = _device()
    xy, m = lens_tensors(lens_xy, lens_m, dev)
    c = to_params(params, mode, exact_recheck=exact_recheck)
    n = int((params["i1"] - params["i0"]) * (params["j1"] - params["j0"]))
    pix = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = new_workspace(params, xy.shape[0], mode, dev)
    L.check(L.lib().rs_ray_pixels(ctypes.byref(c), _ptr(xy), _ptr(m), xy.shape[0], pix.data_ptr(),
                                  workspace.data_ptr(), workspace.numel(), _stream_handle(stream)))
    _hold(stream, xy, m, pix, workspace)
    pix = pix[:n]
    if return_stats:
        return pix, read_stats(workspace, stream)
    return pix


def read_stats(workspace: torch.Tensor, stream=None) -> dict:
    st = L.MapStats()
    L.check(L.lib().rs_read_stats(workspace.data_ptr(), ctypes.byref(st), _stream_handle(stream)))
    return st.as_dict()


def profile_enable(on: bool = True) -> None:
    L.check(L.lib().rs_profile_enable(1 if on else 0))


def profile_read():
    """(kernel milliseconds, launches, interactions) of the deflection launches since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    inter = ctypes.c_double()
    L.check(L.lib().rs_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(inter)))
    return ms.value, n.value, inter.value


def version() -> str:
    return L.lib().rs_version().decode()


def tune(params: dict, lens_xy, lens_m=None, mode: str = "mixed", sample_rays: int = 1 << 22, stream=None) -> dict:
    """Time every thread shape of the deflection kernel on a sample of this map; cache the fastest."""
    dev = _device()
    xy, m = lens_tensors(lens_xy, lens_m, dev)
    c = to_params(params, mode)
    scratch = torch.empty((c.npy, c.npx), dtype=torch.uint32, device=dev)
    ws = new_workspace(params, xy.shape[0], mode, dev)
    r = L.TuneResult()
    L.check(L.lib().rs_tune(ctypes.byref(c), _ptr(xy), _ptr(m), xy.shape[0], scratch.data_ptr(), ws.data_ptr(),
                            ws.numel(), int(sample_rays), _stream_handle(stream), ctypes.byref(r)))
    _hold(stream, xy, m, scratch, ws)
    shapes = [dict(shape=k, rays_per_lane=(r.rays_per_lane[k][0], r.rays_per_lane[k][1]),
                   threads=r.threads[k], ms=r.ms[k],
                   interactions_per_s=r.sample_interactions / (r.ms[k] * 1e-3) if r.ms[k] > 0 else 0.0)
              for k in range(r.n_shapes)]
    return dict(best=r.shape, shapes=shapes, sample_interactions=r.sample_interactions)


def set_shape(shape: int) -> int:
    """Force a thread shape (or -1 for tuned/default); returns the previous setting."""
    prev = ctypes.c_int(0)
    L.check(L.lib().rs_set_shape(int(shape), ctypes.byref(prev)))
    return prev.value


def tune_save(path: str) -> None:
    L.check(L.lib().rs_tune_save(path.encode()))


def tune_load(path: str) -> None:
    L.check(L.lib().rs_tune_load(path.encode()))


class Batch:
    """Device-resident inputs and outputs of a batch of maps, reusable across launches.

    maps: list of (params dict, lens_xy, lens_m or None). All maps share ``mode``.
    """

    def __init__(self, maps, mode: str = "mixed", device=None):
        dev = device or _device()
        self.mode = mode
        self.lenses = [lens_tensors(xy, m, dev) for (_, xy, m) in maps]
        self.params = [p for (p, _, _) in maps]
        self.outs = [torch.empty((int(p["npy"]), int(p["npx"])), dtype=torch.uint32, device=dev)
                     for p in self.params]
        n = len(maps)
        self.reqs = (L.MapRequest * n)()
        for k, (p, (xy, m)) in enumerate(zip(self.params, self.lenses)):
            r = self.reqs[k]
            r.params = to_params(p, mode)
            r.lens_xy = _ptr(xy)
            r.lens_m = _ptr(m)
            r.n_lens = xy.shape[0]
            r.map = self.outs[k].data_ptr()
        nbytes = L.lib().rs_batch_workspace_bytes(self.reqs, n)
        if nbytes == 0:
            L.check(L.RS_EINVAL)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    @property
    def interactions(self) -> int:
        return sum(int((p["i1"] - p["i0"]) * (p["j1"] - p["j0"])) * xy.shape[0]
                   for p, (xy, _) in zip(self.params, self.lenses))

    def run(self, stream=None):
        """Enqueue every map of the batch (asynchronous)."""
        L.check(L.lib().rs_make_maps(self.reqs, len(self.params), self.workspace.data_ptr(),
                                     self.workspace.numel(), _stream_handle(stream)))
        _hold(stream, self.workspace, *self.outs, *(t for pair in self.lenses for t in pair))
        return self.outs

    def tune(self, sample_rays: int = 1 << 20, stream=None) -> dict:
        """Time every thread shape and persistent grid on a band of every map (the maps are
        overwritten) and cache the fastest for batches like this one."""
        r = L.TuneBatchResult()
        L.check(L.lib().rs_tune_batch(self.reqs, len(self.params), self.workspace.data_ptr(), self.workspace.numel(),
                                      int(sample_rays), _stream_handle(stream), ctypes.byref(r)))
        cands = [dict(shape=r.shape[k], rays_per_lane=SHAPES[r.shape[k]], blocks_per_cu=r.blocks_per_cu[k],
                      ms=r.ms[k]) for k in range(r.n)]
        return dict(best=cands[r.best], candidates=cands, sample_interactions=r.sample_interactions)

    def stats(self, stream=None):
        n = len(self.params)
        st = (L.MapStats * n)()
        L.check(L.lib().rs_batch_read_stats(self.workspace.data_ptr(), n, st, _stream_handle(stream)))
        return [s.as_dict() for s in st]


def make_maps(maps, mode: str = "mixed", stream=None, return_stats: bool = False):
    """Build many maps in one persistent launch; returns a list of uint32 [npy, npx] tensors."""
    b = Batch(maps, mode)
    outs = b.run(stream)
    if return_stats:
        return outs, b.stats(stream)
    return outs


class Server:
    """The request loop (continuous batching). Inputs are host arrays; results come back as numpy maps."""

    def __init__(self, hbm_budget_bytes: int = 1 << 30, max_inflight: int = 16, mode: str = "mixed",
                 slice_ms: float = 10.0, starve_s: float = 0.5, max_waiting: int = 0):
        """max_waiting: requests waiting for admission before submit raises RS_EBUSY (0: 4096)."""
        _device()
        cfg = L.ServerCfg(int(hbm_budget_bytes), int(max_inflight), MODES[mode], float(slice_ms), float(starve_s),
                          int(max_waiting))
        h = ctypes.c_void_p()
        L.check(L.lib().rs_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._pending = {}   # ticket -> (host map, keep-alive arrays)
        self.mode = mode

    def submit(self, params: dict, lens_xy, lens_m=None) -> int:
        xy = np.ascontiguousarray(np.asarray(lens_xy, dtype=np.float64).reshape(-1, 2))
        m = None if lens_m is None else np.ascontiguousarray(np.asarray(lens_m, dtype=np.float64).reshape(-1))
        out = np.zeros((int(params["npy"]), int(params["npx"])), dtype=np.uint32)
        c = to_params(params, self.mode)
        t = ctypes.c_uint64()
        L.check(L.lib().rs_server_submit(self._h, ctypes.byref(c), xy.ctypes.data if xy.shape[0] else None,
                                         None if m is None else m.ctypes.data, xy.shape[0], out.ctypes.data,
                                         ctypes.byref(t)))
        self._pending[t.value] = out
        return t.value

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int()
        L.check(L.lib().rs_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        """(map numpy uint32, stats dict, latency seconds); raises RayshootError if cancelled or failed."""
        st = L.MapStats()
        lat = ctypes.c_double()
        rc = L.lib().rs_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(lat))
        out = self._pending.pop(ticket, None)
        L.check(rc)
        return out, st.as_dict(), lat.value

    def cancel(self, ticket: int) -> None:
        L.check(L.lib().rs_server_cancel(self._h, ticket))

    def stats(self) -> dict:
        st = L.ServerStats()
        L.check(L.lib().rs_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            L.lib().rs_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Map statistics (Section 3.1, Accuracy: RMS and K-S assessment; Eq. deltam): dm per pixel,
# count histograms, and the RMS / K-S comparison of two maps.
# ---------------------------------------------------------------------------

def _count_map(t, name="map") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous uint32 device tensor")
    if t.numel() < 1:
        raise ValueError(f"{name} is empty")
    return t


def rays_per_pixel(params: dict) -> float:
    """N_rays of the params' shooting and source grids (Section 3.1)."""
    c = to_params(params, "fp32")
    v = float(L.lib().rs_rays_per_pixel(ctypes.byref(c)))
    if v != v:
        L.check(L.RS_EINVAL)
    return v


def map_max(counts: torch.Tensor, stream=None, out: Optional[torch.Tensor] = None):
    """Largest count of a map. With ``out`` (a 1-element int32 device tensor, read as uint32)
    the call is asynchronous and returns ``out``; otherwise it returns a Python int."""
    _count_map(counts)
    dst = out if out is not None else torch.empty(1, dtype=torch.int32, device=counts.device)
    L.check(L.lib().rs_map_max(counts.data_ptr(), counts.numel(), dst.data_ptr(), _stream_handle(stream)))
    _hold(stream, counts, dst)
    if out is not None:
        return out
    return int(dst.item()) & 0xFFFFFFFF


def histogram(counts: torch.Tensor, max_count: Optional[int] = None, stream=None) -> torch.Tensor:
    """int64 device tensor [max_count + 2]: pixels per count 0..max_count, then pixels above."""
    _count_map(counts)
    if max_count is None:
        max_count = map_max(counts, stream)
    hist = torch.empty(int(max_count) + 2, dtype=torch.int64, device=counts.device)
    L.check(L.lib().rs_map_histogram(counts.data_ptr(), counts.numel(), int(max_count), hist.data_ptr(),
                                     _stream_handle(stream)))
    _hold(stream, counts, hist)
    return hist


def delta_m(counts: torch.Tensor, n_rays: float, stream=None) -> torch.Tensor:
    """float64 device tensor of dm = -2.5 log10(N / N_rays), the map's shape (+inf where N = 0)."""
    _count_map(counts)
    dm = torch.empty(counts.shape, dtype=torch.float64, device=counts.device)
    L.check(L.lib().rs_delta_m(counts.data_ptr(), counts.numel(), float(n_rays), dm.data_ptr(),
                               _stream_handle(stream)))
    _hold(stream, counts, dm)
    return dm


def compare_workspace_bytes(max_a: int, max_b: int) -> int:
    """Workspace bytes of compare_maps for count bounds max_a, max_b."""
    return int(L.lib().rs_compare_workspace_bytes(int(max_a), int(max_b)))


def compare_maps(map_a: torch.Tensor, map_b: torch.Tensor, n_rays_a: float, n_rays_b: Optional[float] = None,
                 max_a: Optional[int] = None, max_b: Optional[int] = None,
                 workspace: Optional[torch.Tensor] = None, stream=None) -> dict:
    """RMS of dm_a - dm_b, K-S statistic D and P(KS), mean magnifications, empty pixels."""
    _count_map(map_a, "map_a")
    _count_map(map_b, "map_b")
    if map_a.numel() != map_b.numel():
        raise ValueError("maps differ in size")
    n_rays_b = n_rays_a if n_rays_b is None else n_rays_b
    if max_a is None:
        max_a = map_max(map_a, stream)
    if max_b is None:
        max_b = map_max(map_b, stream)
    need = compare_workspace_bytes(max_a, max_b)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=map_a.device)
    res = L.CompareResult()
    L.check(L.lib().rs_compare_maps(map_a.data_ptr(), map_b.data_ptr(), map_a.numel(), float(n_rays_a),
                                    float(n_rays_b), int(max_a), int(max_b), workspace.data_ptr(),
                                    workspace.numel(), ctypes.byref(res), _stream_handle(stream)))
    _hold(stream, map_a, map_b, workspace)
    return res.as_dict()
