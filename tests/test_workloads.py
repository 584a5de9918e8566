"""The seeded workload generator against numbers printed in the paper and the config arithmetic."""
import json
import math
import os

import numpy as np

from paper_1005_5198_amd import workloads as w

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_nstar_sigma_sweep_paper_rule():
    """Section 3.1 sigma sweep: the inferred disc rule reproduces 8 of 9 printed N* exactly."""
    g = GOLDEN["nstar_sigma_sweep"]
    got = [w.n_star_for_disc(s, w.paper_rule_radius(s, g["gamma"])) for s in g["sigma"]]
    for s, a, b in zip(g["sigma"], got, g["nstar"]):
        if s == 0.9:
            assert abs(a - b) / b < 5e-4   # printed 41257, rule gives 41267
        else:
            assert a == b, (s, a, b)


def test_nstar_gamma_sweep_paper_rule():
    g = GOLDEN["nstar_gamma_sweep"]
    got = [w.n_star_for_disc(g["sigma"], w.paper_rule_radius(g["sigma"], gm)) for gm in g["gamma"]]
    assert got == g["nstar"]


def test_fig1_nstar():
    g = GOLDEN["fig1_map"]
    assert w.n_star_for_disc(g["sigma"], w.paper_rule_radius(g["sigma"], g["gamma"])) == g["nstar"]
    s = w.paper_point(0.4, 0.0)
    assert s.n_lens == 558


def test_mu_av_printed_values():
    """Eq. (mutheory) against the two worked values printed in Section 3.2."""
    for c in GOLDEN["mu_av_worked"]["cases"]:
        got = 1.0 / ((1.0 - c["sigma"]) ** 2 - c["gamma"] ** 2)
        assert round(got, c["printed_digits"]) == c["mu_av"]
        assert w.mu_av(c["sigma"], c["gamma"]) == got


def test_phi_range():
    g = GOLDEN["phi_range"]
    for key in ("low", "high"):
        e = g[key]
        phi = g["n_flop"] * e["n_pix"] * e["nstar"] * e["n_rays"]
        assert abs(phi - e["phi"]) / e["phi"] < 0.02


def test_configs_arithmetic():
    c0, c1, c2 = w.config0(), w.config1(), w.config2()
    assert c0.n_lens == 462 and c1.n_lens == 462 and c2.n_lens == 17240
    assert c0.interactions == 484_442_112
    assert c1.interactions == 32768 * 32768 * 462
    assert c2.interactions == 1_271_070_720_000
    assert c2.params["sw"] / c2.params["nx"] == 0.0125 and c2.params["sh"] / c2.params["ny"] == 0.0125
    # lenses inside their discs, seeded and reproducible
    for s, r in ((c0, 34.0), (c2, 146.8)):
        assert np.all(np.hypot(s.lens_xy[:, 0], s.lens_xy[:, 1]) <= r)
    assert np.array_equal(w.config0().lens_xy, c0.lens_xy)
    assert not np.array_equal(c0.lens_xy, c1.lens_xy)


def test_config2_shooting_rectangle_matches_eq_square():
    """240 x 48 = 1.2 x Eq. (square) at sigma = 0.8, gamma = 0.3; R = 1.2 x half-diagonal."""
    a, b = w.shooting_sides(0.8, 0.3, 20.0)
    assert math.isclose(1.2 * a, 240.0) and math.isclose(1.2 * b, 48.0)
    assert abs(1.2 * 0.5 * math.hypot(240.0, 48.0) - 146.8) < 0.1


def test_config3_distribution():
    maps = w.config3()
    assert len(maps) == 64
    for s in maps:
        p = s.params
        sigma = p["sigma_star"] + p["sigma_c"]
        assert 0.2 <= p["sigma_star"] <= 0.8 and 0.0 <= p["gamma"] <= 0.4
        assert p["sigma_c"] / sigma <= 0.5 + 1e-12
        assert min(abs(1 - sigma - p["gamma"]), abs(1 - sigma + p["gamma"])) >= 0.1
        assert s.n_lens <= 20000 and p["npx"] in (256, 512, 1024)
        # about 200 rays per pixel received on average: rays ~ 1.44 * 200 * N_pix
        assert 0.9 < s.n_rays / (288.0 * p["npx"] * p["npy"]) < 1.1
    total = sum(s.interactions for s in maps)
    assert 1e13 < total < 5e13


def test_config4_arrivals_are_poisson():
    times, maps = w.config4_arrivals(400, rate_per_s=10.0)
    gaps = np.diff(times)
    assert np.all(gaps >= 0) and abs(gaps.mean() - 0.1) < 0.02
    assert len(maps) == 400


def test_phi_fiducial_scale():
    """Section 2's Phi_fiducial (the cost model Phi): N_FLOP N_pix N* N_rays = 10 x 2500^2 x 1e6 x 500 = 3.1e16."""
    s = w.phi_fiducial()
    assert s.n_lens == 1_000_000
    assert s.params["npx"] == s.params["npy"] == 2500
    assert abs(10 * s.interactions - 10 * 2500 ** 2 * 1e6 * 500) / 3.125e16 < 1e-4
    # the disc radius is the paper rule's for this map side
    assert abs(w.paper_rule_radius(0.45, 0.0, s.params["tw"]) - math.sqrt(1e6 / 0.45)) < 1e-9
    r = np.hypot(s.lens_xy[:, 0], s.lens_xy[:, 1])
    assert r.max() <= math.sqrt(1e6 / 0.45)
