"""The oracle and the host launch planning under sanitizers, on the CPU.

* tests/oracle_driver.c includes oracle/oracle.c whole; built with AddressSanitizer +
  UndefinedBehaviorSanitizer and with ThreadSanitizer (clang), it runs oracle_make_map and
  oracle_ray_pixels on the pins' kinds of input (no lenses, a point lens, masses, random rays,
  a ray on a lens, rays on pixel edges, a window of config 0) on 4 threads, and every output
  must equal the ordinary build's bit for bit, with no sanitizer report.
* tests/plan_driver.cpp runs the runtime's validation and launch planning
  (paper_1005_5198_amd/csrc/plan.cpp) over a table of windows under AddressSanitizer +
  UndefinedBehaviorSanitizer and checks every plan's invariants (whole 32-row bands, queue
  indices below the mark bits, records and bins for every launch, offsets aligned and inside
  the workspace, plans within a fixed scratch).
"""
import ctypes
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1005_5198_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = shutil.which("clang", path="/opt/rocm/llvm/bin") or shutil.which("clang")


def _cases():
    c0 = w.config0()
    yield "c0_window", c0.window(300, 700, 400, 560).params, c0.lens_xy, None
    p = w.make_params(0.0, 0.0, 0.0, (-2.0, -2.0, 4.0, 4.0, 64, 64), (-2.0, -2.0, 4.0, 4.0, 16, 16))
    yield "identity", p, np.zeros((0, 2)), None
    yield "point_lens", p, np.array([[0.0, 0.0]]), None
    # a lens exactly on a grid point (a singular ray) and rays on pixel edges (dyadic grid)
    yield "singular_and_edges", p, np.array([[-0.53125, -0.53125], [0.25, 0.75]]), None
    rng = np.random.default_rng(9)
    q = w.make_params(0.3, 0.1, -0.2, (-6.0, -5.0, 12.0, 10.0, 97, 83), (-4.0, -4.0, 8.0, 8.0, 23, 19))
    yield "masses", q, rng.uniform(-7, 7, size=(37, 2)), rng.uniform(0.1, 3.0, size=37)
    r = dict(q)
    r.update(random_rays=1, seed=11)
    yield "random_rays", r, rng.uniform(-7, 7, size=(29, 2)), None


def _write_input(path, params, xy, m):
    op = oracle._params(params)
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    with open(path, "wb") as f:
        f.write(bytes(op))
        f.write(np.array([xy.shape[0], 0 if m is None else 1], dtype=np.int64).tobytes())
        f.write(xy.tobytes())
        if m is not None:
            f.write(np.ascontiguousarray(m, dtype=np.float64).tobytes())


def _read_output(path, params):
    raw = open(path, "rb").read()
    off = 0

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a
    rc = take(np.int32, 2)
    counts = take(np.uint64, 4)
    npix = int(params["npx"] * params["npy"])
    rays = int((params["i1"] - params["i0"]) * (params["j1"] - params["j0"]))
    mp = take(np.uint32, npix).reshape(int(params["npy"]), int(params["npx"]))
    near = take(np.int64, 2 * int(min(counts[3], 4096))).reshape(-1, 2)
    pix, u, v = take(np.int64, rays), take(np.float64, rays), take(np.float64, rays)
    assert off == len(raw)
    return rc, counts, mp, near, pix, u, v


@pytest.fixture(scope="module", params=["asan_ubsan", "tsan"])
def driver(request, tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("odrv") / f"oracle_{request.param}")
    src = os.path.join(ROOT, "tests", "oracle_driver.c")
    common = ["-std=c11", "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-fno-fast-math", "-ffp-contract=off", "-pthread"]
    if request.param == "asan_ubsan":
        cmd = ["gcc", *common, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    else:
        if CLANG is None:
            pytest.skip("clang not found")
        cmd = [CLANG, *common, "-fsanitize=thread"]
    subprocess.run(cmd + [src, "-o", exe, "-lm"], check=True)
    return exe


@pytest.mark.parametrize("name,params,xy,m", list(_cases()), ids=[c[0] for c in _cases()])
def test_oracle_under_sanitizers_matches(driver, tmp_path, name, params, xy, m):
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, params, xy, m)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    p = subprocess.run([driver, inp, out, "4"], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "Sanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    rc, counts, mp, near, pix, u, v = _read_output(out, params)
    assert rc.tolist() == [0, 0]
    m_ref, st = oracle.make_map(params, xy, m, nthreads=4)
    assert np.array_equal(mp, m_ref)
    assert counts.tolist()[:3] == [st["rays_in_map"], st["rays_out"], st["rays_singular"]]
    assert int(counts[3]) == st["near_edge"]
    assert sorted(map(tuple, near.tolist())) == sorted(st["near_edge_rays"])
    pix_r, u_r, v_r = oracle.ray_pixels(params, xy, m, nthreads=4)
    assert np.array_equal(pix, pix_r)
    assert np.array_equal(u.view(np.uint64), u_r.view(np.uint64))
    assert np.array_equal(v.view(np.uint64), v_r.view(np.uint64))


@pytest.fixture(scope="module")
def plan_results(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("pdrv") / "plan_asan_ubsan")
    csrc = os.path.join(ROOT, "paper_1005_5198_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "plan_driver.cpp"), os.path.join(csrc, "plan.cpp"), "-o", exe],
                   check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and "runtime error" not in p.stderr, p.stderr[-4000:]
    return json.loads(p.stdout)


def test_validation_table(plan_results):
    assert plan_results["validate_wrong"] == []
    assert plan_results["validate_cases"] >= 19


def test_plan_invariants(plan_results):
    assert plan_results["plan_broken"] == []
    assert plan_results["plans"] > 400 and plan_results["plans_within"] > 1000
    assert plan_results["plans_refused"] > 0


def test_config2_plans(plan_results):
    # one launch of 73.7e6 rays: 4 bytes of queue per ray plus the records
    assert plan_results["c2_chunks"] == 1
    assert 4 * 19200 * 3840 <= plan_results["c2_bytes"] < 4 * 19200 * 3840 + (48 << 20)
    # within the 64 MiB scratch of the entry point without allocation: 736-row launches (several
    # launches also hold the 1 MiB list of rays gathered for one exact stage)
    assert plan_results["c2_scratch_chunks"] == 6 and plan_results["c2_scratch_rows"] == 736
