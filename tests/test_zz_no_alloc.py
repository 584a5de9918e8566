"""The entry point without allocation (rs_make_map_noalloc) against rs_make_map (needs an MI355X).

rs_make_map_noalloc runs the same kernels with the library's static per-device scratch
instead of a caller workspace, in launches of as many 32-row bands as that scratch holds.
On the regular grid its map and counters must equal rs_make_map's bit for bit in every
mode; the mixed mode with random rays too. Two calls in a row, the second on a smaller
input, check that what one call leaves in the scratch does not reach the next.
"""
import sys

import numpy as np
import pytest

from paper_1005_5198_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COUNTERS = ("rays_shot", "rays_in_map", "rays_out", "rays_singular", "rays_rechecked")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1005_5198_amd as rs_mod
    return rs_mod


def both(rs, spec, mode, params=None):
    p = params or spec.params
    xy, m = rs.lens_tensors(spec.lens_xy, spec.lens_m)
    ref, st_ref = rs.make_map(p, xy, m, mode=mode, return_stats=True)
    # a stale map in the output: the call must zero it
    out = torch.full_like(ref, 7)
    got, st = rs.make_map_noalloc(p, xy, m, mode=mode, out=out, return_stats=True)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), st_ref, got.cpu().numpy(), st


def check_equal(name, ref, st_ref, got, st, counters=COUNTERS):
    diff = int(np.count_nonzero(ref != got))
    say(f"  {name}: pixels differing {diff}, in map {st['rays_in_map']}, re-checked {st['rays_rechecked']} "
        f"(rs_make_map {st_ref['rays_rechecked']})")
    assert diff == 0
    for k in counters:
        assert st[k] == st_ref[k], (k, st[k], st_ref[k])


def test_two_calls_large_then_small(rs):
    """Config 2 whole (73.7e6 rays, several launches from the 64 MiB scratch), then a
    config-0 window: both equal rs_make_map."""
    from paper_1005_5198_amd import _lib
    c2 = w.config2()
    say(f"noalloc c2 mixed: {c2.n_rays} rays x {c2.n_lens} lenses, scratch {_lib.RS_NOALLOC_SCRATCH_BYTES >> 20} MiB, "
        f"workspace of rs_make_map {rs.workspace_bytes(c2.params, c2.n_lens, 'mixed') >> 20} MiB")
    check_equal("c2 mixed", *both(rs, c2, "mixed"))
    c0 = w.config0().window(100, 900, 37, 701)
    say(f"noalloc c0 window mixed: {c0.n_rays} rays")
    check_equal("c0 window mixed", *both(rs, c0, "mixed"))


@pytest.mark.parametrize("mode", ["fp32", "farfield"])
def test_other_modes(rs, mode):
    c2 = w.config2().window(0, 19200, 1000, 2700)
    say(f"noalloc c2 band {mode}: {c2.n_rays} rays")
    check_equal(f"c2 band {mode}", *both(rs, c2, mode))
    c0 = w.config0()
    check_equal(f"c0 {mode}", *both(rs, c0, mode))


def test_random_rays_mixed(rs):
    c2 = w.config2().window(0, 19200, 0, 640)
    p = dict(c2.params)
    p.update(random_rays=1, seed=2)
    say(f"noalloc c2 random rays mixed: {c2.n_rays} rays")
    # launches of other sizes sort the rays into other bins, so other rays are flagged for
    # the FP64 re-check; the map and the ray counts are the definition's either way
    check_equal("c2 random mixed", *both(rs, c2, "mixed", p),
                counters=("rays_shot", "rays_in_map", "rays_out", "rays_singular"))


def test_masses_and_accumulate(rs):
    c0 = w.config0().window(0, 1024, 0, 300)
    rng = np.random.default_rng(11)
    masses = rng.uniform(0.1, 2.0, c0.n_lens)
    xy, m = rs.lens_tensors(c0.lens_xy, masses)
    ref = rs.make_map(c0.params, xy, m, mode="mixed")
    rs.make_map(c0.params, xy, m, mode="mixed", out=ref, accumulate=True)
    got = rs.make_map_noalloc(c0.params, xy, m, mode="mixed")
    rs.make_map_noalloc(c0.params, xy, m, mode="mixed", out=got, accumulate=True)
    assert np.array_equal(ref.cpu().numpy(), got.cpu().numpy())


def test_too_wide_for_the_scratch_is_refused(rs):
    """One 32-row band of a 2^22-ray-wide mixed window needs 512 MiB of queue: RS_ENOMEM,
    with nothing enqueued."""
    from paper_1005_5198_amd import _lib
    p = w.config0().params.copy()
    p.update(nx=1 << 22, i0=0, i1=1 << 22, j0=0, j1=32)
    xy, m = rs.lens_tensors(w.config0().lens_xy)
    out = torch.zeros((p["npy"], p["npx"]), dtype=torch.uint32, device="cuda")
    with pytest.raises(_lib.RayshootError) as ei:
        rs.make_map_noalloc(p, xy, m, mode="mixed", out=out)
    assert ei.value.code == _lib.RS_ENOMEM
    say("  refused:", ei.value)
    torch.cuda.synchronize()
    assert int(out.sum()) == 0
