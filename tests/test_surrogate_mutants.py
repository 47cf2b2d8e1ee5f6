"""The surrogate oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle/surrogate.py (on the CPU,
in a temporary directory), imports the copy and runs every pin of
test_surrogate_oracle_pins.py against it: at least one pin must fail.
"""
import importlib.util
import os

import pytest

import test_surrogate_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "surrogate.py")

MUTANTS = {
    # Adam (bias-corrected moments)
    "adam: beta2 in the first-moment recurrence": ("m = beta1 * np.asarray(m, np.float64)",
                                                   "m = beta2 * np.asarray(m, np.float64)"),
    "adam: beta1 in the second-moment recurrence": ("v = beta2 * np.asarray(v, np.float64)",
                                                    "v = beta1 * np.asarray(v, np.float64)"),
    "adam: (1 - beta2) weight on the new gradient in m": ("+ (1 - beta1) * g\n", "+ (1 - beta2) * g\n"),
    "adam: first moment corrected with beta2": ("mhat = m / (1 - beta1 ** step)", "mhat = m / (1 - beta2 ** step)"),
    "adam: correction one step late": ("vhat = v / (1 - beta2 ** step)", "vhat = v / (1 - beta2 ** (step + 1))"),
    "adam: correction one step early": ("mhat = m / (1 - beta1 ** step)", "mhat = m / (1 - beta1 ** (step - 1))"),
    "adam: eps inside the square root": ("(np.sqrt(vhat) + eps)", "np.sqrt(vhat + eps)"),
    "adam: gradient not squared": ("(1 - beta2) * g * g", "(1 - beta2) * np.abs(g)"),
    # network
    "gelu derivative sign": ("+ z * np.exp(-0.5 * z * z)", "- z * np.exp(-0.5 * z * z)"),
    "bias gradient averaged again": ("db2 = dz2.sum(axis=0)", "db2 = dz2.mean(axis=0)"),
    "bf16 truncated": ("r = ((u + 0x7FFF + lsb) >> 16) << 16", "r = (u >> 16) << 16"),
    "batch mean dropped": ("dz3 = (p - np.asarray(t, np.float64)) / B", "dz3 = (p - np.asarray(t, np.float64))"),
    # map -> histogram
    "magnification inverted": ("((dx * dy) / (px * py))", "((px * py) / (dx * dy))"),
    "taps not normalised": ("return g / g.sum(), r", "return g, r"),
    "taps of the wrong width": ("g = np.exp(-0.5 * ((k * pixel) / sigma) ** 2)", "g = np.exp(-((k * pixel) / sigma) ** 2)"),
    "natural log for log10": ("np.log10(np.where(mu_s > 0, mu_s, 1.0) / mu_ref)",
                              "np.log(np.where(mu_s > 0, mu_s, 1.0) / mu_ref)"),
    "top bin not clamped": ("b = np.clip(b, 0, nbins - 1)", "b = np.clip(b, 0, nbins)"),
}


def _mutant_module(tmp_path, name):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, name
    path = tmp_path / "surrogate_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("surrogate_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.filterwarnings("ignore::RuntimeWarning")   # a planted mistake may divide by zero
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
