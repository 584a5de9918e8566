"""Map statistics of the accuracy assessment, plain FP64 numpy (test infrastructure only).

Only tests, the smoke check and the bench's CPU-baseline leg import this
module. It shares nothing with the HIP product path.

What the paper defines (Section 3.1, Accuracy; Eq. deltam; Section 2, Eq. mu):
  * the magnification of pixel (i, j) is the number of rays it received
    divided by the average number of rays per pixel without lensing,
    mu_ij = N_ij / N_rays;
  * the change in magnitude of a pixel is  dm_ij = -2.5 log10(mu_ij);
  * two maps are compared by the root-mean-square difference of dm over
    corresponding pixels, and by a two-sample Kolmogorov-Smirnov test on the
    two dm distributions, whose probability P(KS) is the quoted figure.

Readings (the paper is silent on these):
  * a pixel with no rays has mu = 0 and dm = +inf; it takes part in the K-S
    test as a value above every finite one and is left out of the RMS, which
    runs over the pixels where both maps are non-zero (their number is
    returned);
  * P(KS) is the asymptotic Kolmogorov survival function Q_KS(lambda) at
    lambda = (sqrt(n_e) + 0.12 + 0.11 / sqrt(n_e)) D, n_e = n_a n_b / (n_a + n_b)
    (the effective-size correction of Stephens 1970, the usual choice for
    astronomical K-S probabilities);
  * N_rays is the ray density times the pixel area (rays per unit area of the
    shooting grid times the area of one source pixel), Section 3.1.
"""
from __future__ import annotations

import math

import numpy as np


def rays_per_pixel(params) -> float:
    """N_rays: regular-grid ray density times the source-pixel area (Section 3.1, Eq. mu)."""
    density = (params["nx"] / params["sw"]) * (params["ny"] / params["sh"])
    pixel_area = (params["tw"] / params["npx"]) * (params["th"] / params["npy"])
    return density * pixel_area


def magnification(counts, n_rays: float) -> np.ndarray:
    """mu_ij = N_ij / N_rays (Section 2, Eq. mu)."""
    return np.asarray(counts, dtype=np.float64) / float(n_rays)


def delta_m(counts, n_rays: float) -> np.ndarray:
    """dm_ij = -2.5 log10(mu_ij) (Eq. deltam); +inf where the pixel has no rays."""
    mu = magnification(counts, n_rays)
    with np.errstate(divide="ignore"):
        return -2.5 * np.log10(mu)


def rms_delta_m(dm_a, dm_b):
    """Root-mean-square of dm_a - dm_b over the pixels where both are finite.

    Returns (rms, n_used); rms is NaN when no pixel has rays in both maps."""
    a = np.asarray(dm_a, dtype=np.float64).ravel()
    b = np.asarray(dm_b, dtype=np.float64).ravel()
    both = np.isfinite(a) & np.isfinite(b)
    n = int(both.sum())
    if n == 0:
        return math.nan, 0
    d = a[both] - b[both]
    return math.sqrt(float(np.sum(d * d)) / n), n


def ks_statistic(x, y) -> float:
    """Two-sample K-S statistic D = sup_t |F_x(t) - F_y(t)|, F the empirical CDFs.

    The supremum is taken over every sample value of either sample (the only
    places where either CDF jumps); +inf values are ordinary, largest values."""
    xs = np.sort(np.asarray(x, dtype=np.float64).ravel())
    ys = np.sort(np.asarray(y, dtype=np.float64).ravel())
    if xs.size == 0 or ys.size == 0:
        raise ValueError("both samples need at least one value")
    t = np.concatenate([xs, ys])
    fx = np.searchsorted(xs, t, side="right") / xs.size
    fy = np.searchsorted(ys, t, side="right") / ys.size
    return float(np.max(np.abs(fx - fy)))


def kolmogorov_q(lam: float) -> float:
    """Survival function of the Kolmogorov distribution, Q(lam) = P(K > lam).

    For lam >= 1.18 the alternating series 2 sum_j (-1)^(j-1) exp(-2 j^2 lam^2);
    below, 1 minus the Jacobi-transformed series for the CDF,
    sqrt(2 pi)/lam sum_j exp(-(2j-1)^2 pi^2 / (8 lam^2)). Both converge to far
    below 1e-16 within the terms taken."""
    if lam <= 0.0:
        return 1.0
    if lam < 1.18:
        s = 0.0
        for j in range(1, 8):
            s += math.exp(-((2 * j - 1) ** 2) * math.pi ** 2 / (8.0 * lam * lam))
        return 1.0 - math.sqrt(2.0 * math.pi) / lam * s
    s = 0.0
    for j in range(1, 12):
        s += (-1.0) ** (j - 1) * math.exp(-2.0 * j * j * lam * lam)
    return 2.0 * s


def ks_probability(d: float, n_a: int, n_b: int) -> float:
    """P(KS) of statistic d for sample sizes n_a, n_b (Stephens' effective size)."""
    ne = n_a * n_b / (n_a + n_b)
    sq = math.sqrt(ne)
    return kolmogorov_q((sq + 0.12 + 0.11 / sq) * d)


def histogram(counts, max_count: int) -> np.ndarray:
    """Number of pixels with each ray count 0..max_count, then one bin for counts above.

    Divided by the number of pixels, bin c is the probability of magnification
    c / N_rays: the magnification-probability distribution of the map."""
    c = np.asarray(counts).ravel().astype(np.int64)
    h = np.zeros(max_count + 2, dtype=np.int64)
    inside = c <= max_count
    h[: max_count + 1] = np.bincount(c[inside], minlength=max_count + 1)
    h[max_count + 1] = int((~inside).sum())
    return h


def compare_maps(map_a, map_b, n_rays_a: float, n_rays_b: float) -> dict:
    """Everything the accuracy assessment reports for one pair of maps."""
    a = np.asarray(map_a).ravel()
    b = np.asarray(map_b).ravel()
    if a.shape != b.shape:
        raise ValueError("maps differ in size")
    dm_a = delta_m(a, n_rays_a)
    dm_b = delta_m(b, n_rays_b)
    rms, n_both = rms_delta_m(dm_a, dm_b)
    d = ks_statistic(dm_a, dm_b)
    return {
        "rms_dm": rms,
        "n_both": n_both,
        "ks_d": d,
        "ks_p": ks_probability(d, a.size, b.size),
        "mean_mu_a": float(np.mean(magnification(a, n_rays_a))),
        "mean_mu_b": float(np.mean(magnification(b, n_rays_b))),
        "n_zero_a": int((a == 0).sum()),
        "n_zero_b": int((b == 0).sum()),
        "max_a": int(a.max()),
        "max_b": int(b.max()),
    }
