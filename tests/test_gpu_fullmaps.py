"""Whole paper-scale maps against the oracle, every pixel, on the grid and with random rays
(needs an MI355X).

Two kinds of check:
  * fingerprints (default): the whole GPU map of config 1 (1.07e9 rays), config 2 (73.7e6
    rays, 17240 lenses) and config 2 with random rays must have the SHA-256, row sums,
    column sums and ray counts of the oracle's map, stored in tests/golden/fullmaps.json by
    tests/golden/make_fullmaps.py (which calls only the oracle);
  * the oracle run live on the host next to the GPU (default for config 2, about 1.5 min on
    16 host cores; config 1 and random rays only with RS_FULL_ORACLE=1).
The mixed and far-field modes must equal the oracle's map bit for bit (Section 2, Eq. (sigma)
and Eq. (mu_ij)); the oracle's near-edge count (rays within 1e-9 px of an edge) is printed.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1005_5198_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullmaps.json")
FULL = os.environ.get("RS_FULL_ORACLE") == "1"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1005_5198_amd as rs_mod
    oracle.build(force=False)
    return rs_mod


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def case(name):
    spec = w.config1() if name == "c1" else w.config2()
    p = dict(spec.params)
    if name == "c2_random":
        p.update(random_rays=1, seed=2)
    return spec, p


def threads():
    return max(1, min(len(os.sched_getaffinity(0)), 16))


@pytest.mark.parametrize("name,mode", [("c1", "mixed"), ("c1", "farfield"), ("c2", "mixed"),
                                       ("c2", "farfield"), ("c2_random", "mixed")])
def test_whole_map_matches_oracle_fingerprint(rs, golden, name, mode):
    g = golden[name]
    spec, p = case(name)
    say(f"{name} {mode}: {spec.n_rays} rays x {spec.n_lens} lenses; oracle near-edge rays {g['near_edge']}")
    m, st = rs.make_map(p, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
    m = np.ascontiguousarray(m.cpu().numpy(), dtype="<u4")
    sha = hashlib.sha256(m.tobytes()).hexdigest()
    rows = np.flatnonzero(m.sum(axis=1, dtype=np.uint64) != np.asarray(g["row_sums"], dtype=np.uint64))
    cols = np.flatnonzero(m.sum(axis=0, dtype=np.uint64) != np.asarray(g["col_sums"], dtype=np.uint64))
    say(f"  sha256 {sha[:16]} (oracle {g['sha256'][:16]}), rows differing {rows[:8].tolist()}"
        f"{'...' if rows.size > 8 else ''}, columns differing {cols[:8].tolist()}, "
        f"re-checked {st['rays_rechecked']}")
    assert list(m.shape) == g["shape"]
    assert sha == g["sha256"]
    assert st["rays_in_map"] == g["rays_in_map"]
    assert st["rays_out"] == g["rays_out"]
    assert st["rays_singular"] == g["rays_singular"]


def test_config2_whole_map_equals_live_oracle(rs):
    """The config-2 map (1.271e12 interactions) from the oracle on the host cores, every pixel
    compared with the mixed and far-field maps."""
    spec, p = case("c2")
    say(f"c2: oracle on {threads()} threads, {spec.interactions:.3e} interactions")
    t = time.perf_counter()
    m_o, st_o = oracle.make_map(p, spec.lens_xy, spec.lens_m, nthreads=threads())
    dt = time.perf_counter() - t
    say(f"  oracle {dt:.1f} s ({spec.interactions / dt:.3e} ray-lens/s); near-edge rays {st_o['near_edge']}")
    for mode in ("mixed", "farfield"):
        m_g, st_g = rs.make_map(p, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
        diff = int(np.count_nonzero(m_g.cpu().numpy() != m_o))
        say(f"  {mode}: pixels differing {diff}, re-checked {st_g['rays_rechecked']}")
        assert diff == 0
        assert st_g["rays_in_map"] == st_o["rays_in_map"] and st_g["rays_out"] == st_o["rays_out"]


@pytest.mark.skipif(not FULL, reason="set RS_FULL_ORACLE=1 to run the oracle live on these maps "
                                     "(their fingerprints are checked by default)")
@pytest.mark.parametrize("name", ["c1", "c2_random"])
def test_whole_map_equals_live_oracle_opt_in(rs, name):
    spec, p = case(name)
    say(f"{name}: oracle on {threads()} threads, {spec.interactions:.3e} interactions")
    t = time.perf_counter()
    m_o, st_o = oracle.make_map(p, spec.lens_xy, spec.lens_m, nthreads=threads())
    say(f"  oracle {time.perf_counter() - t:.1f} s; near-edge rays {st_o['near_edge']}")
    modes = ("mixed",) if name == "c2_random" else ("mixed", "farfield")
    for mode in modes:
        m_g, st_g = rs.make_map(p, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
        diff = int(np.count_nonzero(m_g.cpu().numpy() != m_o))
        say(f"  {mode}: pixels differing {diff}, re-checked {st_g['rays_rechecked']}")
        assert diff == 0
        assert st_g["rays_in_map"] == st_o["rays_in_map"] and st_g["rays_out"] == st_o["rays_out"]
