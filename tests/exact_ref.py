"""Exact rational evaluation of the lens equation, for tiny inputs.

Independent of both the oracle and the HIP path: Python ``fractions.Fraction``
arithmetic, no rounding anywhere. Used to pin the FP64 oracle on tiny grids
whose parameters are exactly representable (dyadic) numbers.

Lens equation: Section 2, Eq. (sigma). Regular cell-centred ray grid:
Section 3.1. Half-open pixels [p, p+1) in pixel units.
"""
from __future__ import annotations

from fractions import Fraction as F
from typing import Optional, Sequence, Tuple


def frac(x) -> F:
    return F(x)  # exact for any float (binary64 values are dyadic rationals)


def ray_position(p: dict, i: int, j: int) -> Tuple[F, F]:
    x1 = frac(p["sx0"]) + (F(i) + F(1, 2)) * frac(p["sw"]) / p["nx"]
    x2 = frac(p["sy0"]) + (F(j) + F(1, 2)) * frac(p["sh"]) / p["ny"]
    return x1, x2


def source_position(p: dict, lenses: Sequence[Tuple[float, float]], masses: Optional[Sequence[float]],
                    i: int, j: int):
    """Exact (u, v) in pixel units, or None if the ray hits a lens exactly."""
    x1, x2 = ray_position(p, i, j)
    a1 = F(0)
    a2 = F(0)
    for k, (lx, ly) in enumerate(lenses):
        d1 = x1 - frac(lx)
        d2 = x2 - frac(ly)
        r2 = d1 * d1 + d2 * d2
        if r2 == 0:
            return None
        m = F(1) if masses is None else frac(masses[k])
        a1 += m * d1 / r2
        a2 += m * d2 / r2
    g = frac(p["gamma"])
    sc = frac(p["sigma_c"])
    y1 = (1 - g - sc) * x1 - a1
    y2 = (1 + g - sc) * x2 - a2
    u = (y1 - frac(p["tx0"])) * p["npx"] / frac(p["tw"])
    v = (y2 - frac(p["ty0"])) * p["npy"] / frac(p["th"])
    return u, v


def floor_frac(q: F) -> int:
    return q.numerator // q.denominator


def edge_distance(q: F) -> F:
    f = floor_frac(q)
    return min(q - f, f + 1 - q)


def exact_map(p: dict, lenses, masses=None):
    """Exact map over the window: (dict pixel->count, out, singular, min edge distance)."""
    counts = {}
    out = 0
    singular = 0
    min_edge = None
    for j in range(p["j0"], p["j1"]):
        for i in range(p["i0"], p["i1"]):
            r = source_position(p, lenses, masses, i, j)
            if r is None:
                singular += 1
                continue
            u, v = r
            for q in (u, v):
                d = edge_distance(q)
                if min_edge is None or d < min_edge:
                    min_edge = d
            if 0 <= u < p["npx"] and 0 <= v < p["npy"]:
                key = floor_frac(v) * p["npx"] + floor_frac(u)
                counts[key] = counts.get(key, 0) + 1
            else:
                out += 1
    return counts, out, singular, min_edge


def lattice_count_1d(coef: F, s0: F, width: F, n: int, t0: F, tw: F, npix: int):
    """For y = coef * x on a cell-centred grid of n points: per-pixel counts and out count."""
    counts = [0] * npix
    out = 0
    for i in range(n):
        x = s0 + (F(i) + F(1, 2)) * width / n
        u = (coef * x - t0) * npix / tw
        if 0 <= u < npix:
            counts[floor_frac(u)] += 1
        else:
            out += 1
    return counts, out


def near_edge_rays(p: dict, lenses, masses, tol: F):
    """Sorted (i, j) of the window's rays whose exact source position lies within tol
    (strictly) of a pixel edge that matters: both coordinates within [-tol, n + tol] of the
    map, and u or v closer than tol to an integer (the integers 0..n bound the pixels and
    the map). Singular rays are not listed. A ray off the map by more than tol on either
    axis stays out whatever happens on the other, so it is not listed either."""
    tol = F(tol)
    listed = []
    for j in range(p["j0"], p["j1"]):
        for i in range(p["i0"], p["i1"]):
            r = source_position(p, lenses, masses, i, j)
            if r is None:
                continue
            u, v = r
            if not (-tol <= u <= p["npx"] + tol and -tol <= v <= p["npy"] + tol):
                continue
            if edge_distance(u) < tol or edge_distance(v) < tol:
                listed.append((i, j))
    return sorted(listed)
