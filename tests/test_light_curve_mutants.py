"""The light-curve oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU,
in a temporary directory), imports the copy and runs every pin against it:
at least one pin must fail.
"""
import importlib.util
import os

import pytest

import test_light_curve_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "light_curves.py")

MUTANTS = {
    "centre offset dropped": ("ua = (xa - x0) * ipx - 0.5", "ua = (xa - x0) * ipx"),
    "centre offset dropped (points)": ("u = (np.asarray(x, np.float64) - x0) * (1.0 / px) - 0.5",
                                       "u = (np.asarray(x, np.float64) - x0) * (1.0 / px)"),
    "x pixel size for y": ("ipy = 1.0 / py", "ipy = 1.0 / px"),
    "step from the wrong end": ("\n    du = ((xb - xa) * ipx) * inv", "\n    du = ((xb - x0) * ipx) * inv"),
    "fx used for fy": ("out[idx] = r0 + fy * (r1 - r0)", "out[idx] = r0 + fx * (r1 - r0)"),
    "row neighbour for column neighbour": ("r0 = mu_s[j, i] + fx * (mu_s[j, i + 1] - mu_s[j, i])",
                                           "r0 = mu_s[j, i] + fx * (mu_s[j + 1, i] - mu_s[j, i])"),
    "no clamp at the far edge": ("i = min(int(math.floor(uu)), nx - 2)", "i = int(math.floor(uu))"),
    "open hull": ("if not (0.0 <= uu <= nx - 1 and", "if not (0.0 < uu < nx - 1 and"),
    "hull on the map edge": ("0.0 <= vv <= ny - 1)", "-0.5 <= vv <= ny - 0.5)"),
    "sample spacing": ("inv = 1.0 / float(n - 1) if n > 1", "inv = 1.0 / float(n) if n > 1"),
    "strict disk": ("return a * a + b * b <= radius * radius", "return a * a + b * b < radius * radius"),
    "disk row uses px": ("b = float(l) * py", "b = float(l) * px"),
    "disk normalised by its box": ("/ float(len(offs))", "/ float((2 * rx + 1) * (2 * ry + 1))"),
    "disk offsets transposed": ("total += c[ry + l:ry + l + wy, rx + k:rx + k + wx]",
                                "total += c[ry + k:ry + k + wy, rx + l:rx + l + wx]"),
    "norm dropped (Gaussian)": ("np.asarray(counts, np.float64) * norm, size", "np.asarray(counts, np.float64), size"),
    "grid offset by half a pixel": ("return (X0 + rx * Px, Y0 + ry * Py,", "return (X0 + (rx + 0.5) * Px, Y0 + ry * Py,"),
    "Gaussian radius from the other axis": ("math.ceil(3.0 * size / py))", "math.ceil(3.0 * size / px))"),
}


def _mutant_module(tmp_path, name):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, name
    path = tmp_path / "light_curves_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("light_curves_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    mod = _mutant_module(tmp_path, name)
    failed = []
    for pin in pins.PINS:
        try:
            pin(mod)
        except Exception:   # an assertion or a crash both count as caught
            failed.append(pin.__name__)
    assert failed, f"no pin catches the mistake '{name}'"
