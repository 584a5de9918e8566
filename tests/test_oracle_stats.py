"""The map-statistics oracle against its pins, and planted slips against the pins (CPU only).

A mutant is a one-line textual change to a copy of oracle/stats.py, loaded as a
separate module; the committed oracle is never modified."""
import types
import warnings

import pytest

import stats_pins
from oracle import stats as S


@pytest.mark.parametrize("name", sorted(stats_pins.ALL_STATS_PINS))
def test_pin(name):
    stats_pins.ALL_STATS_PINS[name](S)


MUTANTS = {
    "dm_sign": ("return -2.5 * np.log10(mu)", "return 2.5 * np.log10(mu)"),
    "dm_natural_log": ("return -2.5 * np.log10(mu)", "return -2.5 * np.log(mu)"),
    "density_uses_nx_twice": ('density = (params["nx"] / params["sw"]) * (params["ny"] / params["sh"])',
                              'density = (params["nx"] / params["sw"]) * (params["nx"] / params["sh"])'),
    "pixel_area_axes": ('pixel_area = (params["tw"] / params["npx"]) * (params["th"] / params["npy"])',
                        'pixel_area = (params["tw"] / params["npy"]) * (params["th"] / params["npy"])'),
    "rms_over_all_pixels": ("return math.sqrt(float(np.sum(d * d)) / n), n",
                            "return math.sqrt(float(np.sum(d * d)) / a.size), n"),
    "rms_not_rooted": ("return math.sqrt(float(np.sum(d * d)) / n), n", "return float(np.sum(d * d)) / n, n"),
    "ks_mixed_sides": ('fy = np.searchsorted(ys, t, side="right") / ys.size',
                       'fy = np.searchsorted(ys, t, side="left") / ys.size'),
    "ks_wrong_size": ('fy = np.searchsorted(ys, t, side="right") / ys.size',
                      'fy = np.searchsorted(ys, t, side="right") / xs.size'),
    "ks_points_of_one_sample": ("t = np.concatenate([xs, ys])", "t = xs"),
    "q_series_sign": ("s += (-1.0) ** (j - 1) * math.exp(-2.0 * j * j * lam * lam)",
                      "s += math.exp(-2.0 * j * j * lam * lam)"),
    "q_small_lambda_pi": ("s += math.exp(-((2 * j - 1) ** 2) * math.pi ** 2 / (8.0 * lam * lam))",
                          "s += math.exp(-((2 * j - 1) ** 2) * math.pi / (8.0 * lam * lam))"),
    "stephens_dropped": ("return kolmogorov_q((sq + 0.12 + 0.11 / sq) * d)", "return kolmogorov_q(sq * d)"),
    "stephens_sign": ("return kolmogorov_q((sq + 0.12 + 0.11 / sq) * d)",
                      "return kolmogorov_q((sq - 0.12 + 0.11 / sq) * d)"),
    "ne_sum": ("ne = n_a * n_b / (n_a + n_b)", "ne = n_a + n_b"),
    "hist_overflow_dropped": ("h[max_count + 1] = int((~inside).sum())", "pass"),
    "mean_mu_unnormalised": ('"mean_mu_a": float(np.mean(magnification(a, n_rays_a))),',
                             '"mean_mu_a": float(np.mean(a)),'),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_stats_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(S.__file__).read()
    assert src.count(old) == 1, f"mutation anchor not found once for {name}"
    mod = types.ModuleType(f"stats_mutant_{name}")
    mod.__file__ = S.__file__
    exec(compile(src.replace(old, new), f"<stats mutant {name}>", "exec"), mod.__dict__)
    failed = []
    for pin_name, pin in stats_pins.ALL_STATS_PINS.items():
        try:
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                pin(mod)
        except (AssertionError, ValueError, ZeroDivisionError, IndexError):
            failed.append(pin_name)
    assert failed, f"no pin caught stats mutant {name}"
