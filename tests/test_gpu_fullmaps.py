"""Whole paper-scale maps against the oracle, every pixel, on the grid and with random rays
(needs an MI355X and minutes of host CPU).

Skipped unless RS_FULL_ORACLE=1: the oracle takes about 0.5 (config 1) and 1.5 (config 2)
minutes on 16 host cores, too long for the default GPU suite. The windowed and sampled
parity tests cover the same code paths at every size; this is the full-size confirmation.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1005_5198_amd import workloads as w

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(os.environ.get("RS_FULL_ORACLE") != "1",
                                                  reason="set RS_FULL_ORACLE=1 to run whole-map oracle checks")]

torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_whole_map_equals_oracle(rs, name):
    spec = w.CONFIGS[name]()
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    say(f"{name}: oracle on {threads} threads, {spec.interactions:.3e} interactions")
    t = time.perf_counter()
    m_o, st_o = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m, nthreads=threads)
    dt = time.perf_counter() - t
    say(f"  oracle {dt:.1f} s ({spec.interactions / dt:.3e} ray-lens/s); near-edge rays {st_o['near_edge']}")
    for mode in ("mixed", "farfield"):
        m_g, st_g = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
        m_g = m_g.cpu().numpy()
        diff = int(np.count_nonzero(m_g != m_o))
        say(f"  {mode}: pixels differing {diff}, re-checked {st_g['rays_rechecked']}")
        assert diff == 0
        assert st_g["rays_in_map"] == st_o["rays_in_map"] and st_g["rays_out"] == st_o["rays_out"]


def test_whole_random_ray_map_equals_oracle(rs):
    """The config-2 map with random ray positions (seed 2), every pixel: the oracle and the
    kernels each generate the positions from the ray index (Philox4x64-10)."""
    spec = w.config2()
    p = dict(spec.params)
    p.update(random_rays=1, seed=2)
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    say(f"c2 random rays: oracle on {threads} threads, {spec.interactions:.3e} interactions")
    t = time.perf_counter()
    m_o, st_o = oracle.make_map(p, spec.lens_xy, spec.lens_m, nthreads=threads)
    say(f"  oracle {time.perf_counter() - t:.1f} s; near-edge rays {st_o['near_edge']}")
    m_g, st_g = rs.make_map(p, spec.lens_xy, spec.lens_m, mode="mixed", return_stats=True)
    diff = int(np.count_nonzero(m_g.cpu().numpy() != m_o))
    say(f"  mixed: pixels differing {diff}, re-checked {st_g['rays_rechecked']}")
    assert diff == 0
    assert st_g["rays_in_map"] == st_o["rays_in_map"] and st_g["rays_out"] == st_o["rays_out"]
