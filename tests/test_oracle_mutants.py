"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle (on the CPU, in a
temporary directory), builds it, and runs the pins against it: at least one
pin must fail.  The real oracle passes all of them (test_oracle_pins.py).
"""
import os

import numpy as np
import pytest

from oracle import build, shooter
import test_oracle_pins as pins

MUTANTS = {
    "star term sign": ("ax += w * ex;", "ax -= w * ex;"),
    "x/y swapped in star offset": ("double ey = ty - L->ys[k];", "double ey = ty - L->xs[k];"),
    "shear transposed on x": ("double ax = (L->kappa_c + L->gamma1) * tx",
                              "double ax = (L->kappa_c - L->gamma1) * tx"),
    "shear transposed on y": ("double ay = L->gamma2 * tx + (L->kappa_c - L->gamma1) * ty;",
                              "double ay = L->gamma2 * tx + (L->kappa_c + L->gamma1) * ty;"),
    "off-diagonal operand": ("+ L->gamma2 * ty;", "+ L->gamma2 * tx;"),
    "smooth matter dropped": ("double ay = L->gamma2 * tx + (L->kappa_c - L->gamma1) * ty;",
                              "double ay = L->gamma2 * tx + (0.0 - L->gamma1) * ty;"),
    "distance term": ("double r2 = ex * ex + ey * ey;", "double r2 = ex * ex + ex * ey;"),
    "mass dropped": ("double w = L->ms[k] / r2;", "double w = 1.0 / r2;"),
    "Eq. 2 sign": ("*bx = tx - ax;", "*bx = tx + ax;"),
    "cell corner instead of centre": ("double t = (double)idx + 0.5;", "double t = (double)idx;"),
    "closed window": ("u >= 0.0 && u < (double)W->NX", "u >= 0.0 && u <= (double)W->NX"),
    "left edge excluded": ("u >= 0.0 && u < (double)W->NX", "u > 0.0 && u < (double)W->NX"),
    "map transposed": ("return js * W->NX + is;", "return is * W->NY + js;"),
    "rounding instead of floor": ("int64_t is = (int64_t)floor(u);", "int64_t is = (int64_t)(u + 0.5);"),
    "last star skipped": ("for (int64_t k = 0; k < L->n_stars; ++k) {",
                          "for (int64_t k = 0; k + 1 < L->n_stars; ++k) {"),
    # the error scale S that every per-ray beta tolerance is stated against
    "error scale: m/r^2 for m/r": ("s += ms[k] / sqrt(ex * ex + ey * ey);", "s += ms[k] / (ex * ex + ey * ey);"),
    "error scale: sum of |theta| components": ("double s = fmax(fabs(tx), fabs(ty)) + fmax(ax, ay);",
                                               "double s = fabs(tx) + fabs(ty) + fmax(ax, ay);"),
    "error scale: K theta without abs": ("double ay = fabs(gamma2 * tx + (kappa_c - gamma1) * ty);",
                                         "double ay = (gamma2 * tx + (kappa_c - gamma1) * ty);"),
    "error scale: theta without abs": ("fmax(fabs(tx), fabs(ty))", "fmax(tx, ty)"),
    "error scale: star term dropped": ("s += ms[k] / sqrt(", "s += 0.0 * ms[k] / sqrt("),
}


def _pin_suite(lib):
    """Run the pins with the given oracle; return the names that failed."""
    failed = []
    cases = [
        ("point lens", lambda: pins.test_point_lens_enclosed_count(lib, 0.5)),
        ("mass sheet", lambda: pins.test_mass_sheet_plus_point_lens(lib)),
        ("translation", lambda: pins.test_off_centre_star_translation(lib)),
        ("dyadic sheet", lambda: pins.test_dyadic_sheet_is_exact(lib, 0.5, -0.25, 0.1875)),
        ("area law", lambda: pins.test_sheet_area_law(lib)),
        ("pixel edges", lambda: pins.test_pixel_edges_and_window(lib)),
        ("exact brute force", lambda: pins.test_exact_rational_brute_force(lib, 1)),
        ("conservation", lambda: pins.test_map_is_histogram_of_bins(lib)),
        ("mirror", lambda: pins.test_mirror_symmetry(lib)),
        ("bands", lambda: pins.test_band_additivity(lib)),
        ("error scale", lambda: pins.test_error_scale_hand_computed(lib)),
        ("error scale bound", lambda: pins.test_error_scale_bounds_beta(lib)),
    ]
    for name, fn in cases:
        try:
            fn()
        except (AssertionError, ValueError, IndexError):
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(build.SRC).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = shooter.bound(build.build_oracle(out=os.path.join(tmp_path, "libmutant.so"), src=path))
    failed = _pin_suite(lib)
    assert failed, f"no pin caught the mistake: {name}"


def test_real_oracle_passes_suite(oracle_lib):
    assert _pin_suite(shooter.bound(build.LIB)) == []
