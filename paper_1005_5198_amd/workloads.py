"""Seeded synthetic workloads for inverse ray-shooting magnification maps.

This module only draws inputs: lens positions and masses, macro-model
parameters, and the shooting and source grids. It holds none of the
deflection or binning arithmetic, so both the FP64 oracle (tests) and the
HIP path consume exactly the same arrays.

Where the numbers come from:
  * Lens count rule, Section 2, Eq. (nstar): N* = sigma* A / (pi <M>).
    With unit masses and a disc of radius R this is N* = round(sigma* R^2).
  * Lens placement, Section 2 (discussion after Eq. nstar): lenses fill a
    circle whose diameter exceeds the long axis of the "minimum ellipse".
    The paper does not print the radius; two readings are provided:
      - ``paper_rule_radius``: R = 1.5 * (half-diagonal of the L+ x L- shooting
        rectangle) + 2. It reproduces the N* values printed for the sigma and
        gamma sweeps in Section 3.1 (checked in tests/test_workloads.py).
      - the benchmark configurations: R = 1.2 * half-diagonal of a shooting
        rectangle that already carries a 1.2x margin.
  * Spatial distribution (unstated in the paper): area-uniform in the disc,
    r = R sqrt(U1), theta = 2 pi U2, drawn in FP64 with numpy's PCG64.
  * Shooting rectangle, Section 3.2, Eq. (square): L+- = L_map / |1 - sigma +- gamma|;
    the axis that carries 1 - gamma (x1) gets the L_map/|1 - sigma - gamma| side.
  * Regular ray grid, Section 3.1: rays sit on a regular grid; cell-centred
    positions (i + 1/2) * spacing are used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PARAM_KEYS = ("sigma_star", "sigma_c", "gamma",
              "sx0", "sy0", "sw", "sh", "nx", "ny",
              "i0", "i1", "j0", "j1",
              "tx0", "ty0", "tw", "th", "npx", "npy")


@dataclasses.dataclass
class MapSpec:
    """One magnification-map request: macro model, grids, and its lens set."""
    name: str
    params: dict                 # keys: PARAM_KEYS (window defaults to the whole grid)
    lens_xy: np.ndarray          # float64 [N, 2]
    lens_m: Optional[np.ndarray]  # float64 [N] or None (unit masses)

    @property
    def n_lens(self) -> int:
        return int(self.lens_xy.shape[0])

    @property
    def n_rays(self) -> int:
        p = self.params
        return int((p["i1"] - p["i0"]) * (p["j1"] - p["j0"]))

    @property
    def interactions(self) -> int:
        """Ray-lens pairs evaluated by one pass over the window (rays shot x N*)."""
        return self.n_rays * self.n_lens

    def window(self, i0, i1, j0, j1) -> "MapSpec":
        p = dict(self.params)
        p.update(i0=int(i0), i1=int(i1), j0=int(j0), j1=int(j1))
        return MapSpec(self.name + f"[{i0}:{i1},{j0}:{j1}]", p, self.lens_xy, self.lens_m)


def make_params(sigma_star, sigma_c, gamma, shoot, src, window=None) -> dict:
    """shoot = (x0, y0, w, h, nx, ny); src = (x0, y0, w, h, npx, npy)."""
    sx0, sy0, sw, sh, nx, ny = shoot
    tx0, ty0, tw, th, npx, npy = src
    p = dict(sigma_star=float(sigma_star), sigma_c=float(sigma_c), gamma=float(gamma),
             sx0=float(sx0), sy0=float(sy0), sw=float(sw), sh=float(sh), nx=int(nx), ny=int(ny),
             i0=0, i1=int(nx), j0=0, j1=int(ny),
             tx0=float(tx0), ty0=float(ty0), tw=float(tw), th=float(th), npx=int(npx), npy=int(npy))
    if window is not None:
        p.update(i0=int(window[0]), i1=int(window[1]), j0=int(window[2]), j1=int(window[3]))
    return p


def lenses_in_disc(n: int, radius: float, rng: np.random.Generator) -> np.ndarray:
    """n positions area-uniform in a disc of the given radius centred on the origin."""
    u = rng.random((n, 2))
    r = radius * np.sqrt(u[:, 0])
    t = 2.0 * np.pi * u[:, 1]
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1).astype(np.float64)


def n_star_for_disc(sigma_star: float, radius: float, mean_mass: float = 1.0) -> int:
    """Eq. (nstar) with A = pi R^2, rounded to the nearest integer."""
    return int(round(sigma_star * radius * radius / mean_mass))


def shooting_sides(sigma: float, gamma: float, l_map: float) -> tuple:
    """Eq. (square): (side along x1, side along x2) = L_map/|1-sigma-gamma|, L_map/|1-sigma+gamma|."""
    return l_map / abs(1.0 - sigma - gamma), l_map / abs(1.0 - sigma + gamma)


def paper_rule_radius(sigma: float, gamma: float, l_map: float = 20.0) -> float:
    """Lens-disc radius that reproduces the N* printed in Section 3.1 (inferred reading)."""
    lp, lm = shooting_sides(sigma, gamma, l_map)
    return 1.5 * 0.5 * math.hypot(lp, lm) + 2.0


def mu_av(sigma: float, gamma: float) -> float:
    """Eq. (mutheory): theoretical mean magnification of the macro model."""
    return 1.0 / ((1.0 - sigma) ** 2 - gamma ** 2)


# ---------------------------------------------------------------------------
# The named benchmark configurations
# ---------------------------------------------------------------------------

def config0(seed: int = 0) -> MapSpec:
    """sigma*=0.4, gamma=0: 462 unit lenses in R=34; shoot [-20,20)^2 at 1024^2; source [-10,10)^2 at 256^2."""
    rng = np.random.default_rng(seed)
    lens = lenses_in_disc(n_star_for_disc(0.4, 34.0), 34.0, rng)
    p = make_params(0.4, 0.0, 0.0, (-20.0, -20.0, 40.0, 40.0, 1024, 1024),
                    (-10.0, -10.0, 20.0, 20.0, 256, 256))
    return MapSpec("c0_sigma0.4_1024rays_256px", p, lens, None)


def config1(seed: int = 1) -> MapSpec:
    """As config0 with a 32768^2 ray grid and a 1024^2 source map."""
    rng = np.random.default_rng(seed)
    lens = lenses_in_disc(n_star_for_disc(0.4, 34.0), 34.0, rng)
    p = make_params(0.4, 0.0, 0.0, (-20.0, -20.0, 40.0, 40.0, 32768, 32768),
                    (-10.0, -10.0, 20.0, 20.0, 1024, 1024))
    return MapSpec("c1_sigma0.4_32768rays_1024px", p, lens, None)


def config2(seed: int = 2) -> MapSpec:
    """sigma*=0.8, gamma=0.3: 17240 unit lenses in R=146.8; shoot 240x48 at spacing 0.0125; source 1024^2."""
    rng = np.random.default_rng(seed)
    lens = lenses_in_disc(n_star_for_disc(0.8, 146.8), 146.8, rng)
    p = make_params(0.8, 0.0, 0.3, (-120.0, -24.0, 240.0, 48.0, 19200, 3840),
                    (-10.0, -10.0, 20.0, 20.0, 1024, 1024))
    return MapSpec("c2_sigma0.8_gamma0.3_19200x3840rays_1024px", p, lens, None)


def random_map(rng: np.random.Generator, name: str, rays_per_px: float = 200.0,
               max_nstar: int = 20000, src_choices=(256, 512, 1024), l_map: float = 20.0) -> MapSpec:
    """One map from the batched distribution.

    sigma* ~ U[0.2,0.8]; smooth fraction s ~ U[0,0.5] of the total sigma
    (sigma = sigma*/(1-s), sigma_c = sigma - sigma*); gamma ~ U[0,0.4].
    Draws with min|1-sigma+-gamma| < 0.1 or N* > max_nstar are redrawn.
    Shooting sides are 1.2 x Eq. (square); the lens disc radius is 1.2 x the
    shooting half-diagonal. "rays_per_px" is the mean count a source pixel
    receives (so the ray spacing is pix * sqrt(|mu_av| / rays_per_px)).
    """
    while True:
        sstar = rng.uniform(0.2, 0.8)
        s = rng.uniform(0.0, 0.5)
        gamma = rng.uniform(0.0, 0.4)
        sigma = sstar / (1.0 - s)
        sigma_c = sigma - sstar
        if min(abs(1 - sigma - gamma), abs(1 - sigma + gamma)) < 0.1:
            continue
        w1, w2 = shooting_sides(sigma, gamma, l_map)
        w1 *= 1.2
        w2 *= 1.2
        radius = 1.2 * 0.5 * math.hypot(w1, w2)
        nstar = n_star_for_disc(sstar, radius)
        if nstar > max_nstar:
            continue
        break
    npx = int(src_choices[rng.integers(0, len(src_choices))])
    pix = l_map / npx
    spacing = pix * math.sqrt(abs(mu_av(sigma, gamma)) / rays_per_px)
    nx = max(1, int(round(w1 / spacing)))
    ny = max(1, int(round(w2 / spacing)))
    lens = lenses_in_disc(nstar, radius, rng)
    p = make_params(sstar, sigma_c, gamma, (-w1 / 2, -w2 / 2, w1, w2, nx, ny),
                    (-l_map / 2, -l_map / 2, l_map, l_map, npx, npx))
    return MapSpec(name, p, lens, None)


def config3(n_maps: int = 64, seed: int = 3, rays_per_px: float = 200.0) -> List[MapSpec]:
    """The 64-map batch: one child seed per map from SeedSequence(seed)."""
    children = np.random.SeedSequence(seed).spawn(n_maps)
    return [random_map(np.random.default_rng(c), f"c3_map{k:02d}", rays_per_px)
            for k, c in enumerate(children)]


def config4_arrivals(n_requests: int, rate_per_s: float, seed: int = 4,
                     rays_per_px: float = 200.0, src_choices=(256, 512, 1024)):
    """Poisson arrival times (s) and the request maps drawn as in config3."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    times = np.cumsum(gaps) - gaps[0]
    children = np.random.SeedSequence(seed).spawn(n_requests)
    maps = [random_map(np.random.default_rng(c), f"c4_req{k:03d}", rays_per_px,
                       src_choices=src_choices) for k, c in enumerate(children)]
    return times, maps


def paper_point(sigma: float, gamma: float, sigma_c: float = 0.0, n_pix_side: int = 1024,
                n_rays: float = 2000.0, seed: int = 5, l_map: float = 20.0) -> MapSpec:
    """A Section 3.1 parameter point with the paper-rule lens disc and no shooting margin.

    n_rays is the unlensed rays-per-pixel count (ray spacing pix/sqrt(n_rays)).
    """
    rng = np.random.default_rng(seed)
    sigma_star = sigma - sigma_c
    w1, w2 = shooting_sides(sigma, gamma, l_map)
    radius = paper_rule_radius(sigma, gamma, l_map)
    lens = lenses_in_disc(n_star_for_disc(sigma_star, radius), radius, rng)
    pix = l_map / n_pix_side
    spacing = pix / math.sqrt(n_rays)
    nx = int(round(w1 / spacing))
    ny = int(round(w2 / spacing))
    p = make_params(sigma_star, sigma_c, gamma, (-w1 / 2, -w2 / 2, w1, w2, nx, ny),
                    (-l_map / 2, -l_map / 2, l_map, l_map, n_pix_side, n_pix_side))
    return MapSpec(f"paper_sigma{sigma}_gamma{gamma}", p, lens, None)


def phi_fiducial(seed: int = 6, sigma_star: float = 0.45, n_star: int = 1_000_000, n_pix_side: int = 2500,
                 rays_per_px: float = 500.0) -> MapSpec:
    """The Phi_fiducial scale of Section 2 (the cost model Phi): 2500^2 pixels, N* = 1e6 lenses, 500 rays per pixel.

    sigma* = 0.45 in unit-mass lenses, no smooth matter, no shear. The disc holds
    N* = sigma* R^2 lenses; the map side L follows from the paper-rule radius
    R = 1.5 x half-diagonal(L/|1-sigma|, L/|1-sigma|) + 2, and the shooting square is
    the macro model's preimage of the map, side L/|1-sigma|. A pixel receives
    rays_per_px rays on average (mean over the map), so the ray grid holds
    N_pix * rays_per_px rays (the count in the paper's Phi = N_FLOP N_pix N* N_rays):
    55902^2 = 3.125e9 rays and 3.1e15 interactions.
    """
    rng = np.random.default_rng(seed)
    lam = abs(1.0 - sigma_star)
    radius = math.sqrt(n_star / sigma_star)
    l_map = (radius - 2.0) * lam / (1.5 * 0.5 * math.sqrt(2.0))
    side = l_map / lam
    n = int(round(math.sqrt(n_pix_side * n_pix_side * rays_per_px)))
    lens = lenses_in_disc(n_star_for_disc(sigma_star, radius), radius, rng)
    p = make_params(sigma_star, 0.0, 0.0, (-side / 2, -side / 2, side, side, n, n),
                    (-l_map / 2, -l_map / 2, l_map, l_map, n_pix_side, n_pix_side))
    return MapSpec("phi_fiducial_1e6_lenses_2500px", p, lens, None)


CONFIGS = {"c0": config0, "c1": config1, "c2": config2}


def count_map_pair(ny: int, nx: int, n_rays_a: float, n_rays_b: float, seed: int,
                   spike_frac: float = 1e-3, spike_mu=(50.0, 3000.0), log_sigma: float = 0.6):
    """Two uint32 count maps of one synthetic magnification field, as two codes would make them.

    The field: log-normal magnifications (median 1, ln-spread log_sigma) with a
    fraction spike_frac of pixels near caustics (mu log-uniform in spike_mu).
    Each map draws its counts independently, Poisson(mu * N_rays), so low N_rays
    leaves empty pixels and the spikes reach counts far above the median.
    """
    rng = np.random.default_rng(seed)
    mu = rng.lognormal(0.0, log_sigma, size=(ny, nx))
    spikes = rng.random((ny, nx)) < spike_frac
    lo, hi = math.log(spike_mu[0]), math.log(spike_mu[1])
    mu[spikes] = np.exp(rng.uniform(lo, hi, size=int(spikes.sum())))
    a = rng.poisson(mu * n_rays_a).astype(np.uint32)
    b = rng.poisson(mu * n_rays_b).astype(np.uint32)
    return a, b
