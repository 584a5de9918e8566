"""The far-field expansion mode (RS_FARFIELD) on the HIP path vs the FP64 oracle (needs an MI355X).

The mode groups distant lenses into a per-patch FP64 local expansion (the tree
codes' pseudo-lenses with higher multipoles, Section 2, Eq. (hierarchical)),
bounds every ray's error rigorously and re-checks rays near pixel edges in FP64,
so its bar is the mixed mode's: every ray's pixel and the whole map equal the
oracle's, bit for bit.
"""
import sys

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


def check_exact(rs, spec, pixels=True):
    say("farfield exact", spec.name, spec.n_rays, "rays", spec.n_lens, "lenses")
    m_o, st_o = oracle.make_map(spec.params, spec.lens_xy, spec.lens_m)
    m_g, st_g = rs.make_map(spec.params, spec.lens_xy, spec.lens_m, mode="farfield", return_stats=True)
    m_g = m_g.cpu().numpy()
    say(f"  re-checked {st_g['rays_rechecked']} ({st_g['rays_rechecked'] / max(spec.n_rays, 1):.2e})")
    assert np.array_equal(m_g, m_o), f"map differs in {int(np.count_nonzero(m_g != m_o))} pixels"
    assert st_g["rays_in_map"] == st_o["rays_in_map"] and st_g["rays_out"] == st_o["rays_out"]
    assert st_g["rays_singular"] == st_o["rays_singular"] and st_g["rays_shot"] == spec.n_rays
    if pixels:
        pix_o, _, _ = oracle.ray_pixels(spec.params, spec.lens_xy, spec.lens_m)
        pix_g = rs.ray_pixels(spec.params, spec.lens_xy, spec.lens_m, mode="farfield").cpu().numpy()
        assert np.array_equal(pix_g.astype(np.int64), pix_o)
    return st_g


def test_farfield_config0(rs):
    st = check_exact(rs, w.config0())
    assert st["rays_rechecked"] < 1e-3 * 1024 * 1024


def test_farfield_config1_windows(rs):
    s = w.config1()
    for (i0, i1, j0, j1) in ((0, 2048, 0, 96), (15000, 17048, 16300, 16700), (30713, 32768, 32700, 32768)):
        check_exact(rs, s.window(i0, i1, j0, j1))


def test_farfield_config2_windows(rs):
    s = w.config2()
    for (i0, i1, j0, j1) in ((9000, 10000, 1800, 2040), (0, 700, 0, 64), (18500, 19200, 3790, 3840)):
        check_exact(rs, s.window(i0, i1, j0, j1))


def test_farfield_masses(rs):
    s = w.config0()
    rng = np.random.default_rng(23)
    masses = rng.uniform(0.05, 3.0, size=s.n_lens)
    check_exact(rs, w.MapSpec("c0_masses", s.params, s.lens_xy, masses).window(0, 1024, 300, 520))


def test_farfield_crowded_and_singular(rs):
    """600 lenses crowded next to the rays (more than a patch's near list holds: every ray of
    that patch is re-checked), one lens exactly on a ray, one ray far outside."""
    rng = np.random.default_rng(24)
    s = w.config0()
    crowd = np.column_stack([rng.uniform(-0.2, 0.2, 600), rng.uniform(-0.2, 0.2, 600)])
    on_ray = np.array([[-20.0 + (500 + 0.5) * (40.0 / 1024), -20.0 + (512 + 0.5) * (40.0 / 1024)]])
    lenses = np.concatenate([s.lens_xy, crowd, on_ray])
    sub = w.MapSpec("crowded", s.params, lenses, None).window(448, 576, 480, 544)
    check_exact(rs, sub)


def test_farfield_list_overflows(rs):
    """20000 lenses of masses +1 and -1 in a disc of radius 40 over the config-0 grid: more than
    16384 lenses near a group (its list overflows: its super-patches scan every lens), more than
    4096 near a super-patch (the patches scan every lens with both tests), and 25 to 512 within
    four half-diagonals of a patch (more than its record holds: the ray kernel finds them
    itself)."""
    rng = np.random.default_rng(25)
    s = w.config0()
    lenses = w.lenses_in_disc(20000, 40.0, rng)
    masses = np.where(np.arange(20000) % 2 == 0, 1.0, -1.0)
    sub = w.MapSpec("overflows", s.params, lenses, masses).window(448, 576, 480, 544)
    st = check_exact(rs, sub)
    say(f"  re-checked {st['rays_rechecked']}")


def test_farfield_tops(rs):
    """140000 lenses (tops of 4 x 4 groups above the groups) of masses +1 and -1 in a disc of
    radius 1500 around the config-0 grid: most lenses lie beyond four half-diagonals of the
    window's top and enter through its expansion, re-centred three times down to the patch."""
    rng = np.random.default_rng(27)
    s = w.config0()
    n = 140000
    lenses = w.lenses_in_disc(n, 1500.0, rng)
    masses = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    sub = w.MapSpec("tops", s.params, lenses, masses).window(448, 576, 480, 544)
    st = check_exact(rs, sub)
    say(f"  re-checked {st['rays_rechecked']}")


def test_farfield_top_list_overflows(rs):
    """140000 lenses of masses +1 and -1 in a disc of radius 40: every lens lies within four
    half-diagonals of the window's top, so its eight part lists (17500 lenses each) overflow and
    the group scans every lens against the top's test; the group's list and the levels below
    overflow in turn."""
    rng = np.random.default_rng(26)
    s = w.config0()
    n = 140000
    lenses = w.lenses_in_disc(n, 40.0, rng)
    masses = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    sub = w.MapSpec("top overflows", s.params, lenses, masses).window(448, 512, 480, 512)
    st = check_exact(rs, sub)
    say(f"  re-checked {st['rays_rechecked']}")


def test_farfield_config2_full_equals_mixed(rs):
    """The full 19200 x 3840-ray map: the far-field map equals the mixed-mode map (itself the
    oracle's, see the parity tests), and sampled rays equal the oracle's one by one."""
    s = w.config2()
    xy, _ = rs.lens_tensors(s.lens_xy)
    ws = rs.new_workspace(s.params, s.n_lens, "farfield")   # holds the mixed mode's needs too
    mixed = rs.make_map(s.params, xy, None, mode="mixed", workspace=ws)
    ff = rs.make_map(s.params, xy, None, mode="farfield", workspace=ws)
    st = rs.read_stats(ws)
    say(f"config2 farfield: re-checked {st['rays_rechecked']} ({st['rays_rechecked'] / s.n_rays:.2e})")
    assert torch.equal(mixed, ff)
    rng = np.random.default_rng(9)
    for _ in range(4):
        i0 = int(rng.integers(0, 19200 - 64))
        j0 = int(rng.integers(0, 3840 - 32))
        sub = s.window(i0, i0 + 64, j0, j0 + 32)
        pix_o, _, _ = oracle.ray_pixels(sub.params, sub.lens_xy)
        pix_g = rs.ray_pixels(sub.params, xy, None, mode="farfield").cpu().numpy().astype(np.int64)
        assert np.array_equal(pix_g, pix_o)


def test_farfield_phi_fiducial_band_and_samples(rs):
    """1e6 lenses: sampled patches vs the oracle, and a band equal to the direct mixed kernel's."""
    s = w.phi_fiducial()
    xy, _ = rs.lens_tensors(s.lens_xy)
    rng = np.random.default_rng(67)
    for _ in range(2):
        i0 = int(rng.integers(0, s.params["nx"] - 64))
        j0 = int(rng.integers(0, s.params["ny"] - 32))
        sub = s.window(i0, i0 + 64, j0, j0 + 32)
        say("phi_fiducial farfield window", i0, j0)
        pix_o, _, _ = oracle.ray_pixels(sub.params, sub.lens_xy)
        pix_g = rs.ray_pixels(sub.params, xy, None, mode="farfield").cpu().numpy().astype(np.int64)
        assert np.array_equal(pix_g, pix_o)
    j0 = s.params["ny"] // 2
    band = s.window(0, s.params["nx"], j0, j0 + 32)
    a = rs.make_map(band.params, xy, None, mode="farfield")
    b = rs.make_map(band.params, xy, None, mode="mixed")
    assert torch.equal(a, b)
