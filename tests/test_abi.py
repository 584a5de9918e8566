"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
validates arguments before touching a device. No compute calls (no GPU here)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(rs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1005_5198_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 8
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_only_exported_names(lib):
    from paper_1005_5198_amd import _lib
    assert set(_lib.exported_symbols()) <= set(declared_functions())


def test_version(lib):
    from paper_1005_5198_amd import api
    assert "gfx950" in api.version()


def test_workspace_bytes_and_validation(lib):
    from paper_1005_5198_amd import api, workloads as w
    s = w.config2()
    n_mixed = api.workspace_bytes(s.params, s.n_lens, "mixed")
    n_fp32 = api.workspace_bytes(s.params, s.n_lens, "fp32")
    assert n_fp32 < n_mixed
    # the mixed queue holds one launch's rays: whole 32-row bands of the window, at most 2^27 rays
    rows = (1 << 27) // 19200 // 32 * 32
    assert n_mixed >= 4 * min(rows, 3840) * 19200 and n_mixed < 4 * (1 << 27) + 65536
    bad = dict(s.params)
    bad["i1"] = bad["nx"] + 1
    c = api.to_params(bad)
    assert lib.rs_workspace_bytes(ctypes.byref(c), s.n_lens) == 0
    assert b"window" in lib.rs_last_error()


@pytest.mark.parametrize("field,value", [("nx", 0), ("npy", -3), ("sw", 0.0), ("th", float("nan")),
                                         ("j0", -1), ("gamma", float("inf")), ("mode", 7)])
def test_make_map_rejects_before_device_work(lib, field, value):
    from paper_1005_5198_amd import api, _lib, workloads as w
    s = w.config0()
    p = dict(s.params)
    c = api.to_params(p)
    setattr(c, field, value)
    rc = lib.rs_make_map(ctypes.byref(c), None, None, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 30, None)
    assert rc == _lib.RS_EINVAL
    assert lib.rs_last_error()


@pytest.mark.parametrize("npx,npy", [(1 << 31, 1), (1 << 16, 1 << 15), (1 << 32, 1 << 32)])
def test_make_map_rejects_huge_source_grids(lib, npx, npy):
    """2^31 pixels or more is refused, also where npx * npy would wrap around in 64 bits."""
    from paper_1005_5198_amd import api, _lib, workloads as w
    c = api.to_params(w.config0().params)
    c.npx, c.npy = npx, npy
    rc = lib.rs_make_map(ctypes.byref(c), None, None, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 30, None)
    assert rc == _lib.RS_EINVAL
    assert b"2^31 pixels" in lib.rs_last_error()


def test_make_map_rejects_null_outputs(lib):
    from paper_1005_5198_amd import api, _lib, workloads as w
    s = w.config0()
    c = api.to_params(s.params)
    assert lib.rs_make_map(ctypes.byref(c), None, None, 0, None, ctypes.c_void_p(16), 1 << 30, None) == _lib.RS_EINVAL
    assert lib.rs_make_map(ctypes.byref(c), None, None, 5, ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 30,
                           None) == _lib.RS_EINVAL


def test_tune_cache_file_validation(lib, tmp_path):
    from paper_1005_5198_amd import api, _lib
    # lines: kind mode unit n_bucket patch_bucket choice
    for text in ("0 1 1 9 15 77\n",      # shape 13 does not exist
                 "0 1 1 9 15 34\n",      # single maps take no blocks-per-CU part
                 "2 1 1 9 15 1\n",       # kind 2
                 "0 1 1 9 15\n",         # five fields
                 "0 1 1 9 15 1\n1 1 1\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        with pytest.raises(_lib.RayshootError):
            api.tune_load(str(bad))
    good = tmp_path / "good.txt"
    good.write_text("0 1 1 9 15 2\n1 1 0 14 11 49\n")
    api.tune_load(str(good))
    out = tmp_path / "out.txt"
    api.tune_save(str(out))
    text = out.read_text()
    assert "0 1 1 9 15 2" in text and "1 1 0 14 11 49" in text


def test_set_shape_range(lib):
    from paper_1005_5198_amd import api, _lib
    with pytest.raises(_lib.RayshootError):
        api.set_shape(99)
    prev = api.set_shape(2)
    assert api.set_shape(prev) == 2


def test_map_statistics_validation(lib):
    """Argument checks of the map-statistics entry points (nothing reaches a device)."""
    from paper_1005_5198_amd import _lib as L, api, workloads as w
    s = w.config0()
    assert api.rays_per_pixel(s.params) == pytest.approx(4.0, rel=1e-15)
    bad = dict(s.params)
    bad["sw"] = -1.0
    assert math.isnan(lib.rs_rays_per_pixel(ctypes.byref(api.to_params(bad))))
    small = lib.rs_compare_workspace_bytes(10, 20)
    assert small >= 256 + 64 * 1024 + 8 * (12 + 22)
    up = lambda v: (v + 255) // 256 * 256   # histograms of max + 2 uint64, 256-byte aligned
    assert lib.rs_compare_workspace_bytes(1000, 20) - small == up(8 * 1002) - up(8 * 12)
    res = L.CompareResult()
    fake = 1 << 20   # never dereferenced: validation fails first
    assert lib.rs_compare_maps(None, fake, 16, 1.0, 1.0, 4, 4, fake, 1 << 20, ctypes.byref(res), None) == L.RS_EINVAL
    assert b"map_a" in lib.rs_last_error()
    assert lib.rs_compare_maps(fake, fake, 0, 1.0, 1.0, 4, 4, fake, 1 << 20, ctypes.byref(res), None) == L.RS_EINVAL
    assert lib.rs_compare_maps(fake, fake, 16, 0.0, 1.0, 4, 4, fake, 1 << 20, ctypes.byref(res), None) == L.RS_EINVAL
    assert lib.rs_compare_maps(fake, fake, 16, 1.0, 1.0, 4, 4, fake, 100, ctypes.byref(res), None) == L.RS_ENOMEM
    assert lib.rs_compare_maps(fake, fake, 16, 1.0, 1.0, 4, 4, fake + 8, 1 << 20, ctypes.byref(res), None) == L.RS_EINVAL
    assert lib.rs_map_histogram(fake, 16, 0xFFFFFFFF, fake, None) == L.RS_EINVAL
    assert lib.rs_delta_m(fake, 16, float("nan"), fake, None) == L.RS_EINVAL
    assert lib.rs_map_max(fake + 2, 16, fake, None) == L.RS_EINVAL


def test_random_rays_flag_validation(lib):
    """Random rays are accepted by the single-map entry points and refused by batches,
    the server and the tuner before anything reaches a device."""
    from paper_1005_5198_amd import _lib as L, api, workloads as w
    s = w.config2()
    p = dict(s.params)
    p.update(random_rays=1, seed=123)
    c = api.to_params(p)
    assert c.flags & L.RS_RANDOM_RAYS and c.seed == 123
    grid_bytes = api.workspace_bytes(s.params, s.n_lens)
    rand_bytes = lib.rs_workspace_bytes(ctypes.byref(c), s.n_lens)
    # the sorted ray list (index + two FP64 coordinates) of one launch is in the workspace
    assert rand_bytes >= 20 * 19200 * 3840 and rand_bytes > grid_bytes
    req = L.MapRequest(c, 1 << 20, None, s.n_lens, 1 << 21)
    ws = 1 << 22
    assert lib.rs_make_maps(ctypes.byref(req), 1, ws, 1 << 40, None) == L.RS_EINVAL
    assert b"random rays" in lib.rs_last_error()


def test_farfield_mode_validation(lib):
    from paper_1005_5198_amd import _lib as L, api, workloads as w
    s = w.config0()
    c = api.to_params(s.params, "farfield")
    assert c.mode == L.RS_FARFIELD
    # it needs the re-check queue plus the super-patch records and lens lists, which the mixed
    # mode on the regular grid holds too (its far-field re-check stage; its exact-only form does
    # not), a record of 40 + 3 x 24 doubles per 64 x 32-ray patch (expansion, bound terms, near
    # lenses), a 256-byte slot for the ray kernel's patch counter, and per group of 4 x 4
    # super-patches, for each of the 4 blocks that scan its lenses, a record of 36 doubles and a
    # list of 1 + 4096 lens indices
    mixed = api.workspace_bytes(s.params, s.n_lens, "mixed")
    ff = lib.rs_workspace_bytes(ctypes.byref(c), s.n_lens)
    exact = lib.rs_workspace_bytes(ctypes.byref(api.to_params(s.params, "mixed", exact_recheck=True)), s.n_lens)
    n_super = -(-16 // 4) * -(-32 // 4)   # 1024^2 rays: 16 x 32 patches, 4 x 4 per super-patch
    n_patch = 16 * 32
    n_group = 1 * 2                       # 4 x 8 super-patches
    rec_bytes = (40 + 3 * 24) * 8
    a256 = lambda b: -(-b // 256) * 256
    assert ff == mixed + a256(n_patch * rec_bytes) + 256 + a256(n_group * 4 * 36 * 8) + a256(n_group * 4 * 4 * 4097)
    assert ff >= exact + n_super * (36 * 8 + 4 * 4097) + n_patch * rec_bytes
    p = dict(s.params)
    p.update(random_rays=1)
    assert lib.rs_workspace_bytes(ctypes.byref(api.to_params(p, "farfield")), s.n_lens) == 0
    assert b"regular grid" in lib.rs_last_error()
    req = L.MapRequest(c, 1 << 20, None, s.n_lens, 1 << 21)
    assert lib.rs_make_maps(ctypes.byref(req), 1, 1 << 22, 1 << 40, None) == L.RS_EINVAL


def test_map_params_matches_the_generator():
    """The binding's parameter packing equals the input generator's (the same fields and values)."""
    from paper_1005_5198_amd import api, workloads as w
    shoot, src = (-120.0, -24.0, 240.0, 48.0, 19200, 3840), (-10.0, -10.0, 20.0, 20.0, 1024, 1024)
    assert api.map_params(0.8, 0.1, 0.3, shoot, src) == w.make_params(0.8, 0.1, 0.3, shoot, src)
    win = (5, 700, 32, 64)
    assert api.map_params(0.8, 0.1, 0.3, shoot, src, win) == w.make_params(0.8, 0.1, 0.3, shoot, src, win)
    assert api.to_params(api.map_params(0.8, 0.1, 0.3, shoot, src)).npx == 1024


def test_window_wider_than_2_22_refused(lib):
    """A launch holds at least one 32-row band, and a launch's ray index must stay below the
    re-check queue's mark bits (bit 30): windows wider than 2^22 rays are refused."""
    from paper_1005_5198_amd import api, workloads as w
    p = dict(w.config0().params)
    p.update(nx=(1 << 22) + 64, i0=0, i1=(1 << 22) + 1, j0=0, j1=32)
    c = api.to_params(p)
    assert lib.rs_workspace_bytes(ctypes.byref(c), 462) == 0
    assert b"2^22" in lib.rs_last_error()
    p.update(i1=1 << 22)
    c = api.to_params(p)
    n = lib.rs_workspace_bytes(ctypes.byref(c), 462)
    # one band of 32 rows: the queue's largest index is 32 * 2^22 - 1 < 2^30
    assert 4 * 32 * (1 << 22) <= n < (1 << 30)


def test_noalloc_entry_point_rejects_before_device_work(lib):
    """rs_make_map_noalloc validates and plans before it looks up its scratch on the device:
    bad parameters give RS_EINVAL, and a window one 32-row band of which does not fit the
    static scratch gives RS_ENOMEM (the pointers are never dereferenced: nothing is launched)."""
    from paper_1005_5198_amd import api, _lib, workloads as w
    s = w.config0()
    bad = dict(s.params)
    bad["npx"] = 0
    c = api.to_params(bad)
    assert lib.rs_make_map_noalloc(ctypes.byref(c), None, None, 0, None, None, None) == _lib.RS_EINVAL
    c = api.to_params(s.params)
    assert lib.rs_make_map_noalloc(ctypes.byref(c), None, None, 0, None, None, None) == _lib.RS_EINVAL
    assert b"NULL" in lib.rs_last_error()
    wide = dict(s.params)
    wide.update(nx=1 << 22, i0=0, i1=1 << 22, j0=0, j1=64)
    c = api.to_params(wide)
    fake = ctypes.c_void_p(1 << 20)   # an aligned, non-null address that is never used
    rc = lib.rs_make_map_noalloc(ctypes.byref(c), fake, None, 462, fake, None, None)
    assert rc == _lib.RS_ENOMEM
    assert b"scratch" in lib.rs_last_error()
    # the FP32 mode needs no queue: the same window plans within the scratch
    c = api.to_params(wide, "fp32")
    n = lib.rs_workspace_bytes(ctypes.byref(c), 462)
    assert 0 < n <= _lib.RS_NOALLOC_SCRATCH_BYTES


def test_tune_cache_from_environment(tmp_path):
    """RAYSHOOT_TUNE_CACHE is loaded on first use (here: the first save) in a fresh process."""
    import subprocess
    import sys
    cache = tmp_path / "cache.txt"
    cache.write_text("0 1 1 14 15 2\n1 1 1 14 16 35\n")
    out = tmp_path / "out.txt"
    code = ("import sys; sys.path.insert(0, %r); from paper_1005_5198_amd import api; api.tune_save(%r)"
            % (ROOT, str(out)))
    env = dict(os.environ, RAYSHOOT_TUNE_CACHE=str(cache), RAYSHOOT_DEBUG="1")
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr[-2000:]
    text = out.read_text()
    assert "0 1 1 14 15 2" in text and "1 1 1 14 16 35" in text
    assert "[rayshoot] tune cache" in p.stderr
