"""The FP64 oracle against the pins (CPU only)."""
import numpy as np
import pytest

import oracle
import oracle_pins
from paper_1005_5198_amd import workloads as w


@pytest.fixture(scope="module")
def orc():
    oracle.build(force=False)
    return oracle.default()


@pytest.mark.parametrize("name", sorted(oracle_pins.ALL_PINS))
def test_pin(orc, name):
    oracle_pins.ALL_PINS[name](orc)


def test_thread_count_invariance(orc):
    s = w.config0().window(0, 1024, 400, 560)
    m1, s1 = orc.make_map(s.params, s.lens_xy, nthreads=1)
    m8, s8 = orc.make_map(s.params, s.lens_xy, nthreads=8)
    assert np.array_equal(m1, m8) and s1 == s8


def test_windows_sum_to_whole(orc):
    """A map split into ray windows sums exactly to the whole map (resume by windows)."""
    s = w.config0()
    p = dict(s.params)
    p.update(j0=300, j1=420)
    whole, sw = orc.make_map(p, s.lens_xy)
    parts = np.zeros_like(whole)
    out = 0
    for (i0, i1, j0, j1) in ((0, 500, 300, 350), (500, 1024, 300, 350), (0, 1024, 350, 420)):
        q = dict(s.params)
        q.update(i0=i0, i1=i1, j0=j0, j1=j1)
        m, st = orc.make_map(q, s.lens_xy)
        parts += m
        out += st["rays_out"]
    assert np.array_equal(parts, whole) and out == sw["rays_out"]


def test_ray_pixels_agree_with_map(orc):
    s = w.config0().window(100, 900, 500, 540)
    m, st = orc.make_map(s.params, s.lens_xy)
    pix, u, v = orc.ray_pixels(s.params, s.lens_xy)
    hist = np.bincount(pix[pix >= 0], minlength=m.size).reshape(m.shape)
    assert np.array_equal(hist, m)
    assert np.count_nonzero(pix == -1) == st["rays_out"]


def test_near_edge_listed(orc):
    """Rays exactly on pixel edges are reported in the near-edge list."""
    p = w.make_params(0.0, 0.0, 0.0, (-8.0, -4.0, 16.0, 8.0, 64, 32), (-7.875, -3.875, 8.0, 4.0, 32, 16))
    m, st = orc.make_map(p, np.zeros((0, 2)))
    assert st["near_edge"] > 0
    i, j = st["near_edge_rays"][0]
    assert 0 <= i < 64 and 0 <= j < 32


def test_config0_mean_mu_sanity(orc):
    """Sanity only (finite lens disc): config0's mean magnification is near mu_av = 1/(1-sigma)^2."""
    s = w.config0()
    m, st = orc.make_map(s.params, s.lens_xy)
    mean_mu = m.sum() / (256 * 256 * 4)
    assert 0.6 * w.mu_av(0.4, 0.0) < mean_mu < 1.2 * w.mu_av(0.4, 0.0)
    assert st["near_edge"] == 0


def test_invalid_arguments(orc):
    p = w.make_params(0.0, 0.0, 0.0, (-1.0, -1.0, 2.0, 2.0, 8, 8), (-1.0, -1.0, 2.0, 2.0, 4, 4))
    for key, bad in (("nx", 0), ("npx", -1), ("sw", 0.0), ("i1", 9), ("j0", -1)):
        q = dict(p)
        q[key] = bad
        with pytest.raises((RuntimeError, ValueError)):
            orc.make_map(q, np.zeros((0, 2)))
