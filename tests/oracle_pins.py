"""Pins for the FP64 oracle: checks against facts the paper and mathematics fix.

Each pin takes an oracle handle (``oracle.default()`` or a test build) and
raises AssertionError when the oracle disagrees. None of them retypes the
oracle's own formula: they use exact rational arithmetic, closed forms,
symmetries, and the numbers printed in the paper.
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np

import exact_ref
from paper_1005_5198_amd import workloads as w


def _p(sigma_c, gamma, shoot, src, window=None):
    return w.make_params(0.0, sigma_c, gamma, shoot, src, window)


NO_LENS = np.zeros((0, 2))


# ---------------------------------------------------------------------------
# Pin 1: identity. No lenses, no shear, no convergence (Section 2, Eq. (mu_ij):
# without lensing every pixel receives exactly N_rays; Section 3.1 regular grid).
# ---------------------------------------------------------------------------
def pin_identity(orc):
    p = _p(0.0, 0.0, (-20.0, -20.0, 40.0, 40.0, 1024, 1024), (-10.0, -10.0, 20.0, 20.0, 256, 256))
    m, st = orc.make_map(p, NO_LENS)
    assert np.all(m == 4), f"identity map not all 4: min {m.min()} max {m.max()}"
    assert st["rays_out"] == 1024 * 1024 - 4 * 256 * 256, st
    assert st["rays_singular"] == 0
    # pixel = 3 ray spacings: 9 per pixel
    p = _p(0.0, 0.0, (-12.0, -12.0, 24.0, 24.0, 96, 96), (-6.0, -6.0, 12.0, 12.0, 16, 16))
    m, st = orc.make_map(p, NO_LENS)
    assert np.all(m == 9), "identity with pix = 3 spacings"
    assert st["rays_out"] == 96 * 96 - 9 * 256


# ---------------------------------------------------------------------------
# Pin 2: pure convergence and shear (sigma_* = 0). The map is separable:
# map[q][p] = c2[q] * c1[p], each factor a 1-D lattice count done in exact
# rationals. Dyadic parameters make the FP64 evaluation exact, so equality
# is exact, including rays that sit exactly on pixel edges.
# ---------------------------------------------------------------------------
def _separable_case(orc, sigma_c, gamma, shoot, src):
    p = _p(sigma_c, gamma, shoot, src)
    m, st = orc.make_map(p, NO_LENS)
    a1 = 1 - F(gamma) - F(sigma_c)
    a2 = 1 + F(gamma) - F(sigma_c)
    c1, _ = exact_ref.lattice_count_1d(a1, F(shoot[0]), F(shoot[2]), shoot[4], F(src[0]), F(src[2]), src[4])
    c2, _ = exact_ref.lattice_count_1d(a2, F(shoot[1]), F(shoot[3]), shoot[5], F(src[1]), F(src[3]), src[5])
    expect = np.outer(np.array(c2, dtype=np.int64), np.array(c1, dtype=np.int64))
    assert m.shape == expect.shape
    assert np.array_equal(m.astype(np.int64), expect), \
        f"separable lattice mismatch at sigma_c={sigma_c} gamma={gamma}: {int(np.abs(m - expect).sum())}"
    total = shoot[4] * shoot[5]
    assert st["rays_out"] == total - int(expect.sum())


def pin_separable(orc):
    # generic dyadic shear and convergence; some rays land outside the map
    _separable_case(orc, 0.125, 0.25, (-20.0, -10.0, 40.0, 20.0, 320, 160), (-10.0, -10.0, 20.0, 20.0, 80, 80))
    # negative parity along x1 (1 - gamma - sigma_c < 0)
    _separable_case(orc, 0.75, 0.5, (-48.0, -16.0, 96.0, 32.0, 384, 256), (-10.0, -10.0, 20.0, 20.0, 40, 40))
    # rays exactly on pixel edges (half-open convention, including u = 0 and u = npx)
    _separable_case(orc, 0.0, 0.0, (-8.0, -4.0, 16.0, 8.0, 64, 32), (-7.875, -3.875, 8.0, 4.0, 32, 16))
    # non-square grids, different spacings per axis
    _separable_case(orc, 0.25, 0.125, (-20.0, -12.0, 40.0, 24.0, 160, 384), (-9.0, -11.0, 18.0, 22.0, 36, 44))


# ---------------------------------------------------------------------------
# Pin 2b: the mean magnification of the macro model, Eq. (mutheory),
# mu_av = 1 / ((1-sigma)^2 - gamma^2); |mu_av| is the mean count ratio.
# ---------------------------------------------------------------------------
def pin_mean_mu(orc):
    for sigma_c, gamma in ((0.3, 0.2), (0.1, 0.45), (0.55, 0.1)):
        a1 = 1.0 - sigma_c - gamma
        a2 = 1.0 - sigma_c + gamma
        spacing = 0.05
        w1 = 1.3 * 20.0 / abs(a1)
        w2 = 1.3 * 20.0 / abs(a2)
        nx = int(round(w1 / spacing))
        ny = int(round(w2 / spacing))
        p = _p(sigma_c, gamma, (-nx * spacing / 2, -ny * spacing / 2, nx * spacing, ny * spacing, nx, ny),
               (-10.0, -10.0, 20.0, 20.0, 64, 64))
        m, _ = orc.make_map(p, NO_LENS)
        n_rays = (20.0 / 64 / spacing) ** 2
        mean_mu = m.sum() / (64 * 64 * n_rays)
        mu = 1.0 / ((1.0 - sigma_c) ** 2 - gamma ** 2)
        assert abs(mean_mu - abs(mu)) < 0.01 * abs(mu), (sigma_c, gamma, mean_mu, mu)


# ---------------------------------------------------------------------------
# Pin 3: a single point lens (m=1 at the origin, sigma_c = gamma = 0).
# The lens equation is radial: |y| = |r - 1/r|. Rays with |y| < U are exactly
# those with x-(U) < r < x+(U), x+- = (sqrt(U^2+4) +- U)/2, and that image
# area is pi U sqrt(U^2+4). Annulus-averaged magnification matches the
# textbook mu(u) = (u^2+2)/(u sqrt(u^2+4)).
# ---------------------------------------------------------------------------
def pin_point_lens(orc, n=600, half=3.0):
    spacing = 2 * half / n
    pix = 1.0 / 64
    p = _p(0.0, 0.0, (-half, -half, 2 * half, 2 * half, n, n), (-4.0, -4.0, 8.0, 8.0, 512, 512))
    lens = np.array([[0.0, 0.0]])
    pix_id, u, v = orc.ray_pixels(p, lens)
    y1 = u * pix - 4.0
    y2 = v * pix - 4.0
    ymag = np.hypot(y1, y2)
    xs = -half + (np.arange(n) + 0.5) * spacing
    X1, X2 = np.meshgrid(xs, xs)
    r = np.hypot(X1, X2).reshape(-1)
    counts = []
    for U in (0.25, 0.5, 1.0, 1.5, 2.0):
        xp = (math.sqrt(U * U + 4) + U) / 2
        xm = (math.sqrt(U * U + 4) - U) / 2
        ok = (np.abs(ymag - U) > 1e-9) & (np.abs(r - xp) > 1e-9) & (np.abs(r - xm) > 1e-9)
        ok &= np.isfinite(ymag)
        by_map = np.count_nonzero((ymag < U) & ok)
        by_preimage = np.count_nonzero((r > xm) & (r < xp) & ok)
        assert by_map == by_preimage, (U, by_map, by_preimage)
        area = by_map * spacing * spacing
        closed = math.pi * U * math.sqrt(U * U + 4)
        # lattice error is bounded by the boundary length times one spacing
        tol = 2 * math.pi * (xp + xm) * spacing * 1.5 + 4 * spacing * spacing
        assert abs(area - closed) < tol, (U, area, closed)
        counts.append((U, by_map))
    # annulus-averaged magnification vs the analytic mu(u), integrated numerically
    from scipy.integrate import quad

    def mu(s):
        return (s * s + 2) / (s * math.sqrt(s * s + 4))

    for (ua, ca), (ub, cb) in zip(counts, counts[1:]):
        mean_mu = (cb - ca) * spacing * spacing / (math.pi * (ub * ub - ua * ua))
        analytic = quad(lambda s: mu(s) * 2 * math.pi * s, ua, ub)[0] / (math.pi * (ub * ub - ua * ua))
        assert abs(mean_mu - analytic) < 0.03 * analytic, (ua, ub, mean_mu, analytic)


# ---------------------------------------------------------------------------
# Pin 4: the sign of gamma swaps the axes. Reflecting everything across the
# diagonal (x1 <-> x2, all grid parameters swapped) and flipping gamma gives
# the transposed map, bit for bit (the arithmetic is the same, operands swapped).
# ---------------------------------------------------------------------------
def pin_gamma_transpose(orc, seed=11):
    rng = np.random.default_rng(seed)
    lens = rng.uniform(-9, 9, size=(37, 2))
    masses = rng.uniform(0.2, 2.0, size=37)
    p = _p(0.15, 0.3, (-7.0, -5.0, 14.0, 10.0, 140, 100), (-3.0, -4.0, 6.0, 8.0, 48, 64))
    q = _p(0.15, -0.3, (-5.0, -7.0, 10.0, 14.0, 100, 140), (-4.0, -3.0, 8.0, 6.0, 64, 48))
    m1, s1 = orc.make_map(p, lens, masses)
    m2, s2 = orc.make_map(q, lens[:, ::-1].copy(), masses)
    assert np.array_equal(m1, m2.T), "gamma-sign transpose mismatch"
    assert s1["rays_out"] == s2["rays_out"]


# ---------------------------------------------------------------------------
# Pin 5: power-of-two similarity. Doubling every length and quadrupling every
# mass scales every FP64 operation exactly by a power of two, and the
# deflection m (x - x_k)/|x - x_k|^2 doubles with the lengths, so the map is
# bit-identical.
# ---------------------------------------------------------------------------
def pin_similarity(orc, seed=12):
    rng = np.random.default_rng(seed)
    lens = rng.uniform(-12, 12, size=(53, 2))
    masses = np.ones(53)
    p = w.make_params(0.3, 0.05, 0.2, (-8.0, -6.0, 16.0, 12.0, 200, 150), (-5.0, -5.0, 10.0, 10.0, 64, 64))
    m1, s1 = orc.make_map(p, lens, masses)
    for k in (2.0, 0.5):
        q = dict(p)
        for key in ("sx0", "sy0", "sw", "sh", "tx0", "ty0", "tw", "th"):
            q[key] = p[key] * k
        m2, s2 = orc.make_map(q, lens * k, masses * k * k)
        assert np.array_equal(m1, m2), f"similarity x{k} changed the map"
        assert s1["rays_out"] == s2["rays_out"]
    assert m1.sum() > 0


# ---------------------------------------------------------------------------
# Pin 6: ray conservation (every ray is binned, out, or singular).
# ---------------------------------------------------------------------------
def pin_conservation(orc, seed=13):
    rng = np.random.default_rng(seed)
    lens = rng.uniform(-6, 6, size=(29, 2))
    p = w.make_params(0.4, 0.1, 0.2, (-5.0, -5.0, 10.0, 10.0, 123, 77), (-4.0, -4.0, 8.0, 8.0, 33, 29),
                      window=(5, 111, 3, 70))
    m, st = orc.make_map(p, lens)
    assert int(m.sum()) + st["rays_out"] + st["rays_singular"] == (111 - 5) * (70 - 3)


# ---------------------------------------------------------------------------
# Pin 7: brute force in exact rationals on tiny grids, dyadic lens positions.
# ---------------------------------------------------------------------------
def pin_brute_force(orc, seeds=(0, 1, 2, 3)):
    for seed in seeds:
        rng = np.random.default_rng(100 + seed)
        n_l = int(rng.integers(1, 6))
        lens = rng.integers(-40, 40, size=(n_l, 2)) / 8.0 + 1.0 / 64
        masses = None if seed % 2 == 0 else rng.integers(1, 16, size=n_l) / 4.0
        sc = int(rng.integers(0, 4)) / 8.0
        g = int(rng.integers(-4, 5)) / 8.0
        p = _p(sc, g, (-4.0, -3.0, 8.0, 6.0, 16, 16), (-3.0, -2.5, 6.0, 5.0, 12, 10))
        m, st = orc.make_map(p, lens, masses)
        counts, out, sing, min_edge = exact_ref.exact_map(p, [tuple(r) for r in lens],
                                                         None if masses is None else list(masses))
        expect = np.zeros_like(m, dtype=np.int64)
        for key, c in counts.items():
            expect.flat[key] = c
        if min_edge is not None and min_edge > F(1, 10 ** 9):
            assert np.array_equal(m.astype(np.int64), expect), f"brute force mismatch seed {seed}"
            assert st["rays_out"] == out and st["rays_singular"] == sing
            assert st["near_edge"] == 0
        else:
            diff = int(np.abs(m.astype(np.int64) - expect).sum())
            assert diff <= 2 * max(st["near_edge"], 1), f"brute force (near-edge case) seed {seed}"


def pin_singular(orc):
    """A lens exactly on a grid point: that ray is dropped and counted (Eq. (sigma) is singular there)."""
    # grid points at (i + 1/2) * 0.25 - 2: lens at x = (5 + 1/2) * 0.25 - 2 = -0.625
    p = _p(0.0, 0.0, (-2.0, -2.0, 4.0, 4.0, 16, 16), (-2.0, -2.0, 4.0, 4.0, 8, 8))
    lens = np.array([[-0.625, -0.625], [1.3, 0.7]])
    m, st = orc.make_map(p, lens)
    counts, out, sing, _ = exact_ref.exact_map(p, [tuple(r) for r in lens])
    assert sing == 1 and st["rays_singular"] == 1
    pix, _, _ = orc.ray_pixels(p, lens)
    assert pix[5 * 16 + 5] == -2


# ---------------------------------------------------------------------------
# Pin 8: the near-edge list (the rays the mixed-precision comparison may
# exclude). With no lenses and unit macro terms every FP64 operation below is
# exact, so the oracle's list must equal the exact-rational list. A dyadic
# tolerance lets rays sit just inside (d = tol/2), exactly at (d = tol) and
# just outside (d = 2 tol) the tolerance, below (k - d) and above (k + d) the
# edges, on the borders 0 and n of the map, on one axis or both.
# ---------------------------------------------------------------------------
def _edge_grid(du, dv):
    """1-px source pixels over [0, 8)^2 and a 48 x 48 ray grid at spacing 1/4 (unlensed,
    u = x1, v = x2). An axis given an offset d has every fourth ray at k + d for
    k = -1 .. 10 (the others a quarter pixel away); None puts every ray 1/16 px or more
    from an edge; both axes reach beyond the map."""
    def origin(d):
        return -2.0 + 1.0 / 16 if d is None else -1.125 + d
    return _p(0.0, 0.0, (origin(du), origin(dv), 12.0, 12.0, 48, 48), (0.0, 0.0, 8.0, 8.0, 8, 8))


def pin_near_edge(orc):
    tol = 2.0 ** -30
    half, at, twice = 2.0 ** -31, 2.0 ** -30, 2.0 ** -29
    cases = [
        (None, -half, True), (None, -at, False), (None, -twice, False),   # v just below edges
        (None, half, True), (None, at, False), (None, twice, False),      # v just above edges
        (-half, None, True), (half, None, True), (-at, None, False),      # u only
        (half, -half, True), (0.0, None, True), (None, None, False),
    ]
    for du, dv, nonempty in cases:
        p = _edge_grid(du, dv)
        _, st = orc.make_map(p, NO_LENS, near_tol=tol, near_cap=48 * 48)
        expect = exact_ref.near_edge_rays(p, [], None, F(tol))
        assert bool(expect) == nonempty, ("case design", du, dv)
        got = sorted(tuple(int(x) for x in r) for r in st["near_edge_rays"])
        assert st["near_edge"] == len(expect) and got == expect, \
            f"near-edge list differs at du={du} dv={dv}: {st['near_edge']} listed, {len(expect)} expected"
    # the map border at 0 and n is covered: rays at -d and n - d (below), n + d (above)
    p = _edge_grid(None, half)
    rows = {j for _, j in exact_ref.near_edge_rays(p, [], None, F(tol))}
    assert 36 in rows and 0 not in rows       # v = 8 + d listed, v = -1 + d not
    p = _edge_grid(None, -half)
    rows = {j for _, j in exact_ref.near_edge_rays(p, [], None, F(tol))}
    assert 4 in rows and 36 in rows and 40 not in rows   # v = -d and 8 - d listed, 9 - d not


# ---------------------------------------------------------------------------
# Random rays (the GPU code's sampling, Section 3.1): Philox4x64-10 against
# numpy's independent implementation, and the statistics the sampling fixes.
# ---------------------------------------------------------------------------
def _numpy_philox(counter, key):
    """numpy's Philox advances its counter before each block, so start one below."""
    c = [int(x) for x in counter]
    k = 0
    while c[k] == 0 and k < 3:
        c[k] = (1 << 64) - 1
        k += 1
    c[k] = (c[k] - 1) % (1 << 64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


def pin_philox(orc, seed=21):
    rng = np.random.default_rng(seed)
    cases = [([0, 0, 0, 0], [0, 0]), ([(1 << 64) - 1] * 4, [(1 << 64) - 1] * 2)]
    for _ in range(12):
        cases.append(([int(x) for x in rng.integers(0, 1 << 63, 4, dtype=np.uint64)],
                      [int(x) for x in rng.integers(0, 1 << 63, 2, dtype=np.uint64)]))
    for ctr, key in cases:
        got = [int(x) for x in orc.philox4x64(ctr, key)]
        assert got == _numpy_philox(ctr, key), f"philox block differs at counter {ctr} key {key}"


def _random(p, seed):
    q = dict(p)
    q.update(random_rays=1, seed=seed)
    return q


def pin_random_identity(orc):
    """Identity lensing with random rays: every ray lands in the map (positions strictly inside
    the rectangle), the total is exactly the regular grid's, and the per-pixel counts scatter
    like a multinomial draw (chi-square dispersion), where the regular grid has none."""
    from scipy import stats
    shoot, src = (-6.0, -3.0, 12.0, 6.0, 240, 120), (-6.0, -3.0, 12.0, 6.0, 48, 24)
    p = _p(0.0, 0.0, shoot, src)
    grid, _ = orc.make_map(p, NO_LENS)
    assert np.all(grid == 25)
    rnd, st = orc.make_map(_random(p, 7), NO_LENS)
    assert st["rays_out"] == 0 and int(rnd.sum()) == 240 * 120
    chi2 = float(((rnd.astype(np.float64) - 25.0) ** 2).sum() / 25.0)
    dof = rnd.size - 1
    pval = stats.chi2.sf(chi2, dof)
    assert 1e-4 < pval < 1 - 1e-4, f"random-ray counts not multinomial: chi2 {chi2:.1f} on {dof} dof"
    # positions are uniform along each axis (Kolmogorov-Smirnov against U(0,1))
    pix, u, v = orc.ray_pixels(_random(p, 7), NO_LENS)
    assert stats.kstest(u / 48.0, "uniform").pvalue > 1e-4
    assert stats.kstest(v / 24.0, "uniform").pvalue > 1e-4
    # another seed is another drawing, the same seed the same one
    again, _ = orc.make_map(_random(p, 7), NO_LENS)
    other, _ = orc.make_map(_random(p, 8), NO_LENS)
    assert np.array_equal(again, rnd) and not np.array_equal(other, rnd)


def pin_random_wiring(orc):
    """Ray (i, j) takes its uniforms from the block at counter (j nx + i, 0, 0, 0), key (seed, 0):
    under identity lensing u is the ray's first uniform in pixel units (to rounding)."""
    shoot = (-6.0, -3.0, 12.0, 6.0, 240, 120)
    p = _random(_p(0.0, 0.0, shoot, shoot[:4] + (48, 24), window=(17, 20, 33, 35)), 99)
    pix, u, v = orc.ray_pixels(p, NO_LENS)
    for n, (i, j) in enumerate((i, j) for j in range(33, 35) for i in range(17, 20)):
        out = _numpy_philox([j * 240 + i, 0, 0, 0], [99, 0])
        u1 = ((out[0] >> 12) + 0.5) / 2.0 ** 52
        u2 = ((out[1] >> 12) + 0.5) / 2.0 ** 52
        assert abs(u[n] - 48.0 * u1) < 1e-9 and abs(v[n] - 24.0 * u2) < 1e-9, (i, j)


def pin_random_mean_mu(orc):
    """Pure convergence and shear with random rays: rays uniform over the shooting rectangle map
    onto a uniform density |mu_av| times the unlensed one, so the mean count per pixel is
    |mu_av| N_rays up to multinomial noise (five standard deviations)."""
    sigma_c, gamma = 0.25, 0.15
    a1, a2 = 1 - gamma - sigma_c, 1 + gamma - sigma_c
    src = (-4.0, -4.0, 8.0, 8.0, 32, 32)
    # shooting rectangle = preimage of a source square of side 10 (covers the map with margin)
    shoot = (-5.0 / a1, -5.0 / a2, 10.0 / a1, 10.0 / a2, 400, 400)
    p = _random(_p(sigma_c, gamma, shoot, src), 5)
    m, st = orc.make_map(p, NO_LENS)
    frac = (8.0 * 8.0) / (10.0 * 10.0)      # share of the rays whose image lands in the map
    n = 400 * 400
    expect = n * frac
    assert abs(int(m.sum()) - expect) < 5 * math.sqrt(n * frac * (1 - frac))
    assert st["rays_in_map"] + st["rays_out"] == n


def pin_random_vs_grid_lensed(orc, lens_seed=31, ray_seed=13):
    """Lensed map: random ray positions give each pixel its regular-grid count only as a mean,
    with Poisson (multinomial) scatter (Section 3.1), so the standardised residuals
    (random - grid)/sqrt(grid) over well-filled pixels have mean ~0 and variance ~1 (a little
    above 1: the grid's own quadrature error adds to the scatter)."""
    rng = np.random.default_rng(lens_seed)
    lens = rng.uniform(-3.0, 3.0, size=(6, 2))
    shoot, src = (-8.0, -8.0, 16.0, 16.0, 640, 640), (-4.0, -4.0, 8.0, 8.0, 40, 40)
    grid, _ = orc.make_map(_p(0.0, 0.0, shoot, src), lens)
    rnd, _ = orc.make_map(_random(_p(0.0, 0.0, shoot, src), ray_seed), lens)
    g = grid.astype(np.float64)
    sel = g >= 50.0
    z = (rnd.astype(np.float64)[sel] - g[sel]) / np.sqrt(g[sel])
    assert sel.sum() > 1000
    assert abs(z.mean()) < 4.0 / math.sqrt(sel.sum()), f"random-ray mean off the grid map: {z.mean():.3f}"
    assert 0.85 < z.var() < 1.25, f"random-ray scatter not Poisson: variance {z.var():.3f}"


ALL_PINS = {
    "philox": pin_philox,
    "random_identity": pin_random_identity,
    "random_wiring": pin_random_wiring,
    "random_mean_mu": pin_random_mean_mu,
    "random_vs_grid_lensed": pin_random_vs_grid_lensed,
    "identity": pin_identity,
    "separable": pin_separable,
    "mean_mu": pin_mean_mu,
    "point_lens": pin_point_lens,
    "gamma_transpose": pin_gamma_transpose,
    "similarity": pin_similarity,
    "conservation": pin_conservation,
    "brute_force": pin_brute_force,
    "singular": pin_singular,
    "near_edge": pin_near_edge,
}
