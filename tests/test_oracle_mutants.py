"""Pin sensitivity: plausible mistakes planted in copies of the oracle must fail a pin.

Each mutant (15 on the lens equation and the grid, 7 on the random rays, 6 on the
near-edge list) is a one-line textual change to a temporary copy of oracle.c,
compiled on the CPU into a temporary library. The committed oracle is never
modified. The unmutated source must pass every pin (test_oracle_pins.py).
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = {
    "sigma_c_sign": ("const double c1 = (1.0 - p->gamma) - p->sigma_c;",
                     "const double c1 = (1.0 - p->gamma) + p->sigma_c;"),
    "shear_axis_swapped": ("const double c1 = (1.0 - p->gamma) - p->sigma_c;",
                           "const double c1 = (1.0 + p->gamma) - p->sigma_c;"),
    "deflection_power": ("const double f = m / r2;", "const double f = m / sqrt(r2);"),
    "deflection_sign": ("a1 += f * d1;", "a1 -= f * d1;"),
    "dropped_y_term_in_r2": ("const double r2 = d1 * d1 + d2 * d2;", "const double r2 = d1 * d1 + d1 * d1;"),
    "wrong_lens_index": ("const double d2 = x2 - lens_xy[2 * k + 1];", "const double d2 = x2 - lens_xy[2 * k];"),
    "mass_ignored": ("const double m = lens_m ? lens_m[k] : 1.0;", "const double m = 1.0;"),
    "corner_rays": ("*x1 = p->sx0 + ((double)i + 0.5) * (p->sw / (double)p->nx);",
                    "*x1 = p->sx0 + ((double)i) * (p->sw / (double)p->nx);"),
    "spacing_uses_ny": ("(p->sw / (double)p->nx)", "(p->sw / (double)p->ny)"),
    "pixel_size_uses_npx": ("r.v = (y2 - p->ty0) / (p->th / (double)p->npy);",
                            "r.v = (y2 - p->ty0) / (p->th / (double)p->npx);"),
    "closed_low_edge": ("r.u >= 0.0 && r.u < (double)p->npx", "r.u > 0.0 && r.u < (double)p->npx"),
    "closed_high_edge": ("r.v >= 0.0 && r.v < (double)p->npy", "r.v >= 0.0 && r.v <= (double)p->npy"),
    "map_transposed": ("r.pix = (int64_t)floor(r.v) * p->npx + (int64_t)floor(r.u);",
                       "r.pix = (int64_t)floor(r.u) * p->npy + (int64_t)floor(r.v);"),
    "singular_counted_as_out": ("r.pix = RAY_SINGULAR;\n            return r;",
                                "r.pix = RAY_OUT;\n            return r;"),
    "macro_term_dropped": ("const double y2 = c2 * x2 - a2;", "const double y2 = x2 - a2;"),
    "philox_multiplier": ("M0 = 0xD2E7470EE14C6C93ull", "M0 = 0xD2E7470EE14C6C95ull"),
    "philox_key_not_bumped": ("k1 += W1;", "k1 += 0;"),
    "philox_output_words": ("c2 = hi0 ^ c3 ^ k1;", "c2 = hi0 ^ c1 ^ k1;"),
    "uniform_53_bits": ("const double u1 = ((double)(out[0] >> 12) + 0.5) * 0x1p-52;",
                        "const double u1 = ((double)(out[0] >> 11) + 0.5) * 0x1p-52;"),
    "uniform_axis_extent": ("*x2 = p->sy0 + u2 * p->sh;", "*x2 = p->sy0 + u2 * p->sw;"),
    "uniform_reused": ("const double u2 = ((double)(out[1] >> 12) + 0.5) * 0x1p-52;",
                       "const double u2 = ((double)(out[0] >> 12) + 0.5) * 0x1p-52;"),
    "counter_transposed": ("(uint64_t)j * (uint64_t)p->nx + (uint64_t)i", "(uint64_t)i * (uint64_t)p->ny + (uint64_t)j"),
    "near_edge_one_sided": ("const double d = fmin(c - f, f + 1.0 - c);", "const double d = c - f;"),
    "near_edge_closed_tol": ("return d < tol;", "return d <= tol;"),
    "near_edge_u_only": ("return near_edge_1d(r->u, p->npx, tol) || near_edge_1d(r->v, p->npy, tol);",
                         "return near_edge_1d(r->u, p->npx, tol);"),
    "near_edge_v_range_ignored": ("if (!in_u || !in_v)\n        return 0;", "if (!in_u)\n        return 0;"),
    "near_edge_upper_border_open": ("r->u <= (double)p->npx + tol;", "r->u < (double)p->npx;"),
    "near_edge_lower_border_open": ("const int in_v = r->v >= -tol", "const int in_v = r->v >= 0.0"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found for {name}"
    mutated = src.replace(old, new, 1)
    path = tmp_path / "oracle_mut.c"
    path.write_text(mutated)
    lib = oracle.build(force=True, src=str(path), out=str(tmp_path / f"liboracle_{name}.so"),
                       extra_flags=("-w",))
    orc = oracle.load(lib)
    failed = []
    for pin_name, pin in oracle_pins.ALL_PINS.items():
        try:
            pin(orc)
        except (AssertionError, RuntimeError):
            failed.append(pin_name)
    assert failed, f"no pin caught mutant {name}"
