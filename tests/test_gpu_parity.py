"""HIP path vs the FP64 oracle on the same seeded inputs (needs an MI355X).

Tolerances (from the method's definition of the count map):
  * RS_MIXED: every ray's pixel and the whole uint32 map equal the oracle's,
    bit for bit. The oracle's near-edge list (rays within 1e-9 px of an edge)
    is reported alongside.
  * RS_FP32: at most 1e-4 of the rays may land in a different pixel than the
    oracle's; the relative L1 map error is reported.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_1005_5198_amd import workloads as w

pytestmark = pytest.mark.gpu

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


def gpu_map(rs, spec, mode):
    out, st = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
    return out.cpu().numpy(), st


def gpu_pix(rs, spec, mode):
    pix, st = rs.ray_pixels(spec.params, spec.lens_xy, spec.lens_m, mode=mode, return_stats=True)
    return pix.cpu().numpy().astype(np.int64), st


def check_mixed_exact(rs, spec):
    say("mixed-exact", spec.name, spec.n_rays, "rays", spec.n_lens, "lenses")
    m_o, st_o = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m)
    m_g, st_g = gpu_map(rs, spec, "mixed")
    say("  oracle near-edge rays:", st_o["near_edge"], " re-checked on GPU:", st_g["rays_rechecked"],
        f"({st_g['rays_rechecked'] / max(spec.n_rays, 1):.4%})")
    assert np.array_equal(m_g, m_o), f"map differs in {int(np.count_nonzero(m_g != m_o))} pixels"
    assert st_g["rays_in_map"] == st_o["rays_in_map"]
    assert st_g["rays_out"] == st_o["rays_out"]
    assert st_g["rays_singular"] == st_o["rays_singular"]
    assert st_g["rays_shot"] == spec.n_rays
    return st_g


def check_pixels(rs, spec, fp32_budget=1e-4):
    say("pixels", spec.name)
    pix_o, _, _ = oracle.ray_pixels(spec.params, spec.lens_xy, spec.lens_m)
    pix_m, _ = gpu_pix(rs, spec, "mixed")
    assert np.array_equal(pix_m, pix_o), f"mixed: {int(np.count_nonzero(pix_m != pix_o))} rays differ"
    pix_f, _ = gpu_pix(rs, spec, "fp32")
    changed = np.count_nonzero(pix_f != pix_o) / max(len(pix_o), 1)
    say(f"  fp32 changed-ray fraction {changed:.3e}")
    assert changed <= fp32_budget
    return changed


def test_config0_mixed_bit_exact(rs):
    st = check_mixed_exact(rs, w.config0())
    assert st["rays_rechecked"] < 0.05 * 1024 * 1024


def test_config0_fp32_map_and_pixels(rs):
    s = w.config0()
    m_o, _ = oracle.make_map(s.params, s.lens_xy)
    m_f, st = gpu_map(rs, s, "fp32")
    rel_l1 = np.abs(m_f.astype(np.int64) - m_o.astype(np.int64)).sum() / m_o.sum()
    say(f"config0 fp32 relative L1 {rel_l1:.3e}")
    assert st["rays_rechecked"] == 0
    assert rel_l1 < 1e-3
    check_pixels(rs, s)


def test_config1_windows(rs):
    s = w.config1()
    for (i0, i1, j0, j1) in ((0, 2048, 0, 96), (15000, 17048, 16300, 16700), (30713, 32768, 32700, 32768)):
        sub = s.window(i0, i1, j0, j1)
        check_mixed_exact(rs, sub)
        check_pixels(rs, sub)


def test_config2_windows(rs):
    s = w.config2()
    for (i0, i1, j0, j1) in ((9000, 10000, 1800, 2040), (0, 700, 0, 64), (18500, 19200, 3790, 3840)):
        sub = s.window(i0, i1, j0, j1)
        check_mixed_exact(rs, sub)
        check_pixels(rs, sub)


def test_config2_full_map_sampled(rs):
    """Full 19200 x 3840-ray map in the launch configuration the benchmark times:
    conservation, determinism, and sampled rays checked one by one against the oracle."""
    s = w.config2()
    say("config2 full map, mixed")
    xy, m = rs.lens_tensors(s.lens_xy)
    ws = rs.new_workspace(s.params, s.n_lens, "mixed")
    out1 = rs.make_map(s.params, xy, None, mode="mixed", workspace=ws)
    st = rs.read_stats(ws)
    out2 = rs.make_map(s.params, xy, None, mode="mixed", workspace=ws)
    st2 = rs.read_stats(ws)
    a, b = out1.cpu().numpy(), out2.cpu().numpy()
    assert np.array_equal(a, b) and st == st2
    assert st["rays_in_map"] + st["rays_out"] + st["rays_singular"] == s.n_rays
    assert int(a.sum()) == st["rays_in_map"]
    say(f"  in-map {st['rays_in_map']}, re-checked {st['rays_rechecked']} "
        f"({st['rays_rechecked'] / s.n_rays:.3%}), against every lens {st['rays_rechecked_direct']}")
    # the whole map equals the one whose flagged rays all take the definition's exact sequence
    exact = rs.make_map(s.params, xy, None, mode="mixed", exact_recheck=True)
    assert torch.equal(out1, exact)
    assert st["rays_rechecked_direct"] < 0.02 * st["rays_rechecked"]
    # sampled rays: a 64 x 16 window at seeded random places, each ray vs the oracle
    rng = np.random.default_rng(7)
    for _ in range(6):
        i0 = int(rng.integers(0, 19200 - 64))
        j0 = int(rng.integers(0, 3840 - 16))
        sub = s.window(i0, i0 + 64, j0, j0 + 16)
        pix_o, _, _ = oracle.ray_pixels(sub.params, sub.lens_xy)
        pix_m, _ = gpu_pix(rs, sub, "mixed")
        assert np.array_equal(pix_m, pix_o)


@pytest.mark.parametrize("random_rays", [False, True])
def test_config1_full_map_staged_equals_exact(rs, random_rays):
    """The 1.07e9-ray map runs as several launches (8 on the grid, 16 with random rays), each
    with its own queue and, on the grid, its own super-patch records: the staged re-check gives
    the same map as the exact sequence for every flagged ray."""
    s = w.config1()
    p = dict(s.params)
    if random_rays:
        p.update(random_rays=1, seed=13)
    say("config1 full map, random" if random_rays else "config1 full map, grid")
    xy, _ = rs.lens_tensors(s.lens_xy)
    a, st = rs.make_map(p, xy, None, mode="mixed", return_stats=True)
    b, st_x = rs.make_map(p, xy, None, mode="mixed", return_stats=True, exact_recheck=True)
    say(f"  re-checked {st['rays_rechecked']}, against every lens {st['rays_rechecked_direct']}")
    assert torch.equal(a, b)
    assert st["rays_rechecked"] == st_x["rays_rechecked"] > 10000
    assert st["rays_rechecked_direct"] < 0.02 * st["rays_rechecked"]
    assert st["rays_in_map"] + st["rays_out"] + st["rays_singular"] == s.n_rays


def test_windows_sum_to_full_map(rs):
    """Ray windows are exact partial maps: their sum equals the full map (checkpoint/resume)."""
    s = w.config0()
    full, _ = gpu_map(rs, s, "mixed")
    xy, _ = rs.lens_tensors(s.lens_xy)
    acc = None
    for (j0, j1) in ((0, 333), (333, 700), (700, 1024)):
        sub = s.window(0, 1024, j0, j1)
        acc = rs.make_map(sub.params, xy, None, mode="mixed", out=acc, accumulate=acc is not None)
    assert np.array_equal(acc.cpu().numpy(), full)


EDGE_CASES = {
    # name: (sigma_c, gamma, shoot, src, window, n_lens, masses)
    "no_lenses_identity": (0.0, 0.0, (-20.0, -20.0, 40.0, 40.0, 1024, 1024), (-10.0, -10.0, 20.0, 20.0, 256, 256), None, 0, False),
    "ragged_window": (0.1, 0.2, (-6.0, -5.0, 12.0, 10.0, 301, 173), (-4.0, -4.0, 8.0, 8.0, 37, 53), (3, 298, 5, 170), 57, False),
    "single_ray": (0.0, 0.1, (-2.0, -2.0, 4.0, 4.0, 9, 9), (-3.0, -3.0, 6.0, 6.0, 5, 5), (4, 5, 4, 5), 7, False),
    "masses": (0.05, 0.15, (-8.0, -8.0, 16.0, 16.0, 257, 255), (-6.0, -6.0, 12.0, 12.0, 64, 48), None, 131, True),
    "negative_parity": (0.7, 0.5, (-30.0, -12.0, 60.0, 24.0, 600, 240), (-8.0, -8.0, 16.0, 16.0, 64, 64), None, 200, False),
    "one_lens_many_tiles_of_rays": (0.0, 0.0, (-3.0, -3.0, 6.0, 6.0, 700, 500), (-4.0, -4.0, 8.0, 8.0, 128, 128), None, 1, False),
    "lens_count_not_multiple_of_tile": (0.2, 0.0, (-10.0, -10.0, 20.0, 20.0, 200, 200), (-5.0, -5.0, 10.0, 10.0, 40, 40), None, 2051, False),
}


@pytest.mark.parametrize("case", sorted(EDGE_CASES))
def test_edge_cases(rs, case):
    sc, g, shoot, src, window, n, masses = EDGE_CASES[case]
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    lens = rng.uniform(-12, 12, size=(n, 2)) if n else np.zeros((0, 2))
    mm = rng.uniform(0.1, 3.0, size=n) if masses else None
    p = w.make_params(0.3, sc, g, shoot, src, window)
    spec = w.MapSpec(case, p, lens, mm)
    check_mixed_exact(rs, spec)
    check_pixels(rs, spec, fp32_budget=2e-3 if case == "single_ray" else 1e-4)


def test_shared_reciprocal_range_guards(rs):
    """The FP32 loop shares one reciprocal between four rays (or two, outside the four-ray
    range) through the product of their r^2. A lens beyond 1e9 (a product of two could
    overflow) flags every block, and a patch under 1e-6 across (it could underflow) is
    flagged whole; a tile with a lens beyond 8192 of a patch, or a patch under 1e-4 across,
    sums with two-ray reciprocals instead. Every map still equals the oracle's, in both the
    mixed and the FP32 mode."""
    rng0 = np.random.default_rng(37)
    # one far lens (beyond the four-ray range, well inside 1e9) in the first tile of 2000
    lens = np.concatenate([[[3.0e5, -2.0e5]], rng0.uniform(-9, 9, size=(1999, 2))])
    p = w.make_params(0.3, 0.1, 0.2, (-6.0, -5.0, 12.0, 10.0, 300, 200), (-4.0, -4.0, 8.0, 8.0, 40, 40))
    spec = w.MapSpec("lens_beyond_quad_range", p, lens, None)
    check_mixed_exact(rs, spec)
    check_pixels(rs, spec, fp32_budget=1e-4)
    # patches 64 x 32 rays of 1e-6 x 1e-6: half-diagonal about 4e-5, two-ray path, not flagged
    small = w.make_params(0.3, 0.0, 0.1, (0.25, 0.5, 1.28e-4, 6.4e-5, 128, 64), (-100.0, -100.0, 200.0, 200.0, 64, 64))
    spec = w.MapSpec("small_patch", small, rng0.uniform(-3, 3, size=(25, 2)), None)
    st = check_mixed_exact(rs, spec)
    assert st["rays_rechecked"] < 128 * 64
    rng = np.random.default_rng(31)
    lens = np.concatenate([rng.uniform(-9, 9, size=(40, 2)), [[2.0e9, 1.0]]])
    p = w.make_params(0.3, 0.1, 0.2, (-6.0, -5.0, 12.0, 10.0, 160, 96), (-4.0, -4.0, 8.0, 8.0, 40, 40))
    st = check_mixed_exact(rs, w.MapSpec("far_lens", p, lens, None))
    assert st["rays_rechecked"] == 160 * 96
    tiny = w.make_params(0.3, 0.0, 0.1, (0.25, 0.5, 2e-8, 1e-8, 128, 64), (-100.0, -100.0, 200.0, 200.0, 64, 64))
    st = check_mixed_exact(rs, w.MapSpec("tiny_patch", tiny, rng.uniform(-3, 3, size=(25, 2)), None))
    assert st["rays_rechecked"] == 128 * 64 and st["rays_in_map"] > 0


def test_shoot_map_signature(rs):
    """shoot_map (model and grids given directly) gives the oracle's map, with and without masses."""
    s = w.config0()
    shoot = (-20.0, -20.0, 40.0, 40.0, 1024, 1024)
    src = (-10.0, -10.0, 20.0, 20.0, 256, 256)
    assert rs.map_params(0.4, 0.0, 0.0, shoot, src) == s.params
    m_o, _ = oracle.make_map(s.params, s.lens_xy)
    got = rs.shoot_map(s.lens_xy, None, 0.4, 0.0, 0.0, shoot, src).cpu().numpy()
    assert np.array_equal(got, m_o)
    masses = np.full(s.n_lens, 0.5)
    m_o2, _ = oracle.make_map(s.params, s.lens_xy, masses)
    got2 = rs.shoot_map(s.lens_xy, masses, 0.4, 0.0, 0.0, shoot, src).cpu().numpy()
    assert np.array_equal(got2, m_o2)


def test_empty_window(rs):
    s = w.config0().window(10, 10, 0, 1024)
    m_g, st = gpu_map(rs, s, "mixed")
    assert m_g.sum() == 0 and st["rays_shot"] == 0


def test_singular_ray_on_lens(rs):
    """A lens exactly on a grid point: the ray is re-checked and counted as singular."""
    p = w.make_params(0.0, 0.0, 0.0, (-2.0, -2.0, 4.0, 4.0, 16, 16), (-2.0, -2.0, 4.0, 4.0, 8, 8))
    lens = np.array([[-0.625, -0.625], [1.3, 0.7]])
    spec = w.MapSpec("singular", p, lens, None)
    st = check_mixed_exact(rs, spec)
    assert st["rays_singular"] == 1
    pix, _ = gpu_pix(rs, spec, "mixed")
    assert pix[5 * 16 + 5] == -2


def test_gamma_transpose_on_gpu(rs):
    """Pin 4 through the HIP path: the mixed map is bit-exact, so the symmetry holds on the GPU."""
    rng = np.random.default_rng(11)
    lens = rng.uniform(-9, 9, size=(37, 2))
    p = w.make_params(0.3, 0.15, 0.3, (-7.0, -5.0, 14.0, 10.0, 140, 100), (-3.0, -4.0, 6.0, 8.0, 48, 64))
    q = w.make_params(0.3, 0.15, -0.3, (-5.0, -7.0, 10.0, 14.0, 100, 140), (-4.0, -3.0, 8.0, 6.0, 64, 48))
    m1, _ = gpu_map(rs, w.MapSpec("a", p, lens, None), "mixed")
    m2, _ = gpu_map(rs, w.MapSpec("b", q, lens[:, ::-1].copy(), None), "mixed")
    assert np.array_equal(m1, m2.T)


def test_invalid_arguments_raise(rs):
    from paper_1005_5198_amd._lib import RayshootError, RS_EINVAL, RS_ENOMEM
    s = w.config0()
    bad = dict(s.params)
    bad["npx"] = 0
    with pytest.raises(RayshootError) as e:
        rs.make_map(bad, s.lens_xy)
    assert e.value.code == RS_EINVAL
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RayshootError) as e:
        rs.make_map(s.params, s.lens_xy, workspace=small)
    assert e.value.code == RS_ENOMEM


def test_exact_only_recheck_matches_two_stage(rs):
    """The two re-check paths (bounded FP64 stage + exact stage, or exact only) give the same map,
    and both equal the oracle's."""
    s = w.config2().window(4000, 5200, 1000, 1240)
    m_o, _ = oracle.make_map(s.params, s.lens_xy)
    a, sa = rs.make_map(s.params, s.lens_xy, mode="mixed", return_stats=True)
    b, sb = rs.make_map(s.params, s.lens_xy, mode="mixed", return_stats=True, exact_recheck=True)
    say(f"re-checked {sa['rays_rechecked']} (two-stage) / {sb['rays_rechecked']} (exact only)")
    assert sa["rays_rechecked"] == sb["rays_rechecked"] > 0
    assert np.array_equal(a.cpu().numpy(), m_o) and np.array_equal(b.cpu().numpy(), m_o)
    pa = rs.ray_pixels(s.params, s.lens_xy, mode="mixed").cpu().numpy()
    pb = rs.ray_pixels(s.params, s.lens_xy, mode="mixed", exact_recheck=True).cpu().numpy()
    assert np.array_equal(pa, pb)


def test_far_field_recheck_stage(rs):
    """The mixed mode's first re-check stage (each queued ray from its super-patch's FP64
    expansion plus the listed lenses) places almost every queued ray; the map and every ray's
    pixel still equal the oracle's and the exact-only re-check's, with unit masses and with
    masses."""
    s = w.config2().window(4000, 5200, 1000, 1240)
    rng = np.random.default_rng(21)
    for masses in (None, rng.uniform(0.2, 1.8, size=s.n_lens)):
        spec = w.MapSpec("far-recheck", s.params, s.lens_xy, masses)
        m_o, _ = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m)
        a, sa = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode="mixed", return_stats=True)
        b, sb = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode="mixed", return_stats=True,
                            exact_recheck=True)
        say(f"masses={masses is not None}: re-checked {sa['rays_rechecked']}, "
            f"of which against every lens {sa['rays_rechecked_direct']}")
        assert sa["rays_rechecked"] == sb["rays_rechecked"] > 1000
        assert sb["rays_rechecked_direct"] == sb["rays_rechecked"]
        assert sa["rays_rechecked_direct"] < 0.01 * sa["rays_rechecked"]
        assert np.array_equal(a.cpu().numpy(), m_o) and np.array_equal(b.cpu().numpy(), m_o)
        pix_o, _, _ = oracle.ray_pixels(spec.params, spec.lens_xy, spec.lens_m)
        pa = rs.ray_pixels(spec.params, spec.lens_xy, spec.lens_m, mode="mixed").cpu().numpy()
        assert np.array_equal(pa.astype(np.int64), pix_o)


def test_far_field_recheck_list_overflow(rs):
    """5000 light lenses inside four half-diagonals of every super-patch: the super-patch lists
    overflow, the far-field stage places nothing, and the FP64 stages over every lens give the
    oracle's map."""
    rng = np.random.default_rng(22)
    lens = w.lenses_in_disc(5000, 5.0, rng)
    mm = rng.uniform(0.0005, 0.0015, size=5000)
    p = w.make_params(0.064, 0.1, 0.2, (-3.0, -2.0, 6.0, 4.0, 300, 200), (-3.0, -2.0, 6.0, 4.0, 120, 80))
    spec = w.MapSpec("overflow", p, lens, mm)
    st = check_mixed_exact(rs, spec)
    say(f"  re-checked {st['rays_rechecked']}, against every lens {st['rays_rechecked_direct']}")
    assert st["rays_rechecked"] > 0
    assert st["rays_rechecked_direct"] == st["rays_rechecked"]


@pytest.mark.parametrize("mode", ["mixed", "farfield"])
def test_exact_stage_gathered_over_launches_and_its_overflow(rs, mode):
    """A map of two launches (8192 x 16400 rays) whose every 33rd column lands exactly on a pixel
    edge (one massless lens: no deflection, y = x; pixels 33/64 wide, rays 1/64 apart): no bound
    can place those 4.1e6 rays, so they all reach the exact stage. The first 65536 are gathered
    over both launches and run after the last one, the rest with their own launch; the map and
    the counts equal the oracle's."""
    nx, ny = 8192, 16400                       # 2^27 + 16 x 8192 rays: two launches
    shoot = (-64.0 - 0.5 / 64, -128.0, 128.0, ny / 64.0, nx, ny)   # x = i/64 - 64, y = (j + 1/2)/64 - 128
    src = (-64.0, -128.0, 132.0, 256.25, 256, 8200)                 # 33/64 x 1/32 pixels
    p = w.make_params(0.0, 0.0, 0.0, shoot, src)
    spec = w.MapSpec("edges", p, np.array([[1000.0, 1000.0]]), np.array([0.0]))
    m_o, st_o = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m)
    m_g, st_g = gpu_map(rs, spec, mode)
    on_edge = len(range(0, nx, 33)) * ny
    say(f"{mode}: re-checked {st_g['rays_rechecked']}, rays on an edge {on_edge}")
    assert st_g["rays_rechecked"] >= on_edge > 65536
    assert np.array_equal(m_g, m_o), f"map differs in {int(np.count_nonzero(m_g != m_o))} pixels"
    assert st_g["rays_in_map"] == st_o["rays_in_map"] == nx * ny
    assert st_g["rays_out"] == st_o["rays_out"] == 0


def test_batch_far_field_stage_list_overflow(rs):
    """A batch whose first map's super-patch lists overflow (5000 lenses within reach of every
    super-patch) next to an ordinary map: the overflowing map's flagged rays all take the stage
    over every lens, the other map's almost none, and both maps equal the oracle's."""
    rng = np.random.default_rng(23)
    lens = w.lenses_in_disc(5000, 5.0, rng)
    mm = rng.uniform(0.0005, 0.0015, size=5000)
    dense = w.MapSpec("overflow", w.make_params(0.064, 0.1, 0.2, (-3.0, -2.0, 6.0, 4.0, 300, 200),
                                                (-3.0, -2.0, 6.0, 4.0, 120, 80)), lens, mm)
    plain = w.config2().window(2000, 2900, 600, 800)
    outs, stats = rs.make_maps([(x.params, x.lens_xy, x.lens_m) for x in (dense, plain)], mode="mixed",
                               return_stats=True)
    for x, o, st in zip((dense, plain), outs, stats):
        say("batch", x.name, st)
        m_o, _ = oracle.make_map(x.params, x.lens_xy, x.lens_m)
        assert np.array_equal(o.cpu().numpy(), m_o), x.name
    assert stats[0]["rays_rechecked"] > 0 and stats[0]["rays_rechecked_direct"] == stats[0]["rays_rechecked"]
    assert stats[1]["rays_rechecked"] > 1000
    assert stats[1]["rays_rechecked_direct"] < 0.02 * stats[1]["rays_rechecked"]


def test_every_shape_gives_the_same_maps(rs):
    """All thread shapes cover the same ray patch, so each ray's arithmetic is the same:
    FP32 maps are bit-identical across shapes, and mixed maps equal the oracle for every shape."""
    s = w.config2().window(7000, 8300, 2000, 2200)
    m_o, _ = oracle.make_map(s.params, s.lens_xy)
    xy, _ = rs.lens_tensors(s.lens_xy)
    fp32_maps = []
    try:
        for shape in range(4):
            rs.set_shape(shape)
            say("shape", shape)
            fp32_maps.append(rs.make_map(s.params, xy, mode="fp32").cpu().numpy())
            assert np.array_equal(rs.make_map(s.params, xy, mode="mixed").cpu().numpy(), m_o)
    finally:
        rs.set_shape(-1)
    for m in fp32_maps[1:]:
        assert np.array_equal(m, fp32_maps[0])


def test_tuner_picks_and_persists(rs, tmp_path):
    s = w.config0()
    res = rs.tune(s.params, s.lens_xy, mode="mixed", sample_rays=1 << 18)
    say("tune:", res)
    assert 0 <= res["best"] < len(res["shapes"])
    assert all(sh["ms"] > 0 for sh in res["shapes"])
    assert res["shapes"][res["best"]]["ms"] == min(sh["ms"] for sh in res["shapes"])
    path = str(tmp_path / "tune.txt")
    rs.tune_save(path)
    rs.tune_load(path)
    lines = [l.split() for l in open(path).read().splitlines() if l.strip()]
    assert lines and all(len(l) == 6 for l in lines)
    assert any(l[0] == "0" and int(l[5]) == res["best"] for l in lines)


def test_batch_tuner_picks_and_maps_stay_exact(rs, tmp_path):
    """The batch tuner times every thread shape and persistent grid on a band of every map;
    the batch then runs with its choice, and the maps still equal the single maps (mixed:
    the oracle's too)."""
    specs = _batch_specs()
    items = [(x.params, x.lens_xy, x.lens_m) for x in specs]
    b = rs.Batch(items, mode="mixed")
    res = b.tune(sample_rays=1 << 16)
    say("batch tune:", res["best"], len(res["candidates"]), "candidates")
    assert len(res["candidates"]) == 12 and res["sample_interactions"] > 0
    assert all(c["ms"] > 0 for c in res["candidates"])
    assert res["best"]["ms"] == min(c["ms"] for c in res["candidates"])
    outs = b.run()
    for x, o in zip(specs, outs):
        single = rs.make_map(x.params, x.lens_xy, x.lens_m, mode="mixed").cpu().numpy()
        assert np.array_equal(o.cpu().numpy(), single), x.name
    path = str(tmp_path / "tune.txt")
    rs.tune_save(path)
    lines = [l.split() for l in open(path).read().splitlines() if l.strip()]
    assert any(l[0] == "1" for l in lines)


def _batch_specs():
    rng = np.random.default_rng(21)
    specs = [w.config0().window(100, 900, 200, 700), w.config2().window(9000, 9700, 1800, 1960)]
    lens = rng.uniform(-12, 12, size=(131, 2))
    specs.append(w.MapSpec("masses", w.make_params(0.3, 0.05, 0.15, (-8.0, -8.0, 16.0, 16.0, 257, 255),
                                                   (-6.0, -6.0, 12.0, 12.0, 64, 48)), lens,
                           rng.uniform(0.1, 3.0, size=131)))
    specs.append(w.MapSpec("negpar", w.make_params(0.3, 0.7, 0.5, (-30.0, -12.0, 60.0, 24.0, 600, 240),
                                                   (-8.0, -8.0, 16.0, 16.0, 64, 64)),
                           rng.uniform(-12, 12, size=(200, 2)), None))
    specs.append(w.MapSpec("nolens", w.make_params(0.0, 0.0, 0.0, (-2.0, -2.0, 4.0, 4.0, 40, 40),
                                                   (-1.0, -1.0, 2.0, 2.0, 10, 10)), np.zeros((0, 2)), None))
    specs.append(w.config1().window(15000, 16100, 16300, 16400))
    return specs


def test_batch_matches_single_and_oracle(rs):
    """Every map of a batch equals its single-map result (both modes) and the oracle (mixed)."""
    specs = _batch_specs()
    items = [(s.params, s.lens_xy, s.lens_m) for s in specs]
    for mode in ("mixed", "fp32"):
        outs, stats = rs.make_maps(items, mode=mode, return_stats=True)
        for s, o, st in zip(specs, outs, stats):
            say("batch", mode, s.name, st)
            single, st1 = rs.make_map(s.params, s.lens_xy, s.lens_m, mode=mode, return_stats=True)
            assert np.array_equal(o.cpu().numpy(), single.cpu().numpy()), f"{s.name} {mode}"
            for key in ("rays_in_map", "rays_out", "rays_singular", "rays_shot"):
                assert st[key] == st1[key], (s.name, key)
            if mode == "mixed":
                # a batch mixing unit and general masses bounds unit-mass maps with the general
                # constant, so it may re-check more rays; the maps stay identical
                assert st["rays_rechecked"] >= st1["rays_rechecked"]
                # the far-field stage places almost every flagged ray in a batch too
                assert st["rays_rechecked_direct"] <= st["rays_rechecked"]
                if st["rays_rechecked"] > 1000:
                    assert st["rays_rechecked_direct"] < 0.02 * st["rays_rechecked"], s.name
                if s.n_rays * s.n_lens < 3e9:
                    m_o, _ = oracle.make_map(s.params, s.lens_xy, s.lens_m)
                    assert np.array_equal(o.cpu().numpy(), m_o)


def _delay(stream, seconds=0.2):
    """Queue a bounded spin on the stream, so that work queued after it starts late."""
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(seconds * 2.4e9))


def test_side_stream_temporaries_stay_alive(rs):
    """make_map and make_maps on a stream other than the current one, with lens copies and
    workspaces made inside the call: while that stream is held back, the current stream
    allocates and overwrites memory; the maps must still equal the oracle's."""
    s = torch.cuda.Stream()
    spec = w.config0().window(0, 1024, 200, 840)
    m_o, _ = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m)
    ws_bytes = rs.workspace_bytes(spec.params, spec.n_lens, "mixed")
    _delay(s)
    out = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode="mixed", stream=s)
    junk = [torch.full((ws_bytes,), 255, dtype=torch.uint8, device="cuda"),
            torch.full((spec.n_lens * 2,), 1e30, dtype=torch.float64, device="cuda")]
    specs = [w.config0().window(0, 512, 0, 512), w.config0().window(300, 1024, 100, 700)]
    _delay(s)
    outs = rs.make_maps([(x.params, x.lens_xy, x.lens_m) for x in specs], mode="mixed", stream=s)
    junk += [torch.full((8 << 20,), 255, dtype=torch.uint8, device="cuda") for _ in range(4)]
    s.synchronize()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), m_o)
    for x, o in zip(specs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.make_map(x.params, x.lens_xy, x.lens_m)[0]), x.name
    del junk

