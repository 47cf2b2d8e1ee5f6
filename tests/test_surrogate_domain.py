"""The surrogate's domain test (host logic; no GPU): a query is the
network's only inside the training box and near a training example."""
import math

import numpy as np

from paper_1703_09707_amd import surrogate as S


def _grid_with_hole():
    g = np.stack(np.meshgrid(*[np.linspace(-1.0, 1.0, 9)] * 4, indexing="ij"), -1).reshape(-1, 4)
    hole = np.all(np.abs(g) <= 0.3, axis=1)   # no examples in the central cube
    return g[~hole]


def test_domain_box_and_holes():
    pts = _grid_with_hole()
    d = S.Domain.fit(pts)
    assert np.allclose(d.lo, -1.0) and np.allclose(d.hi, 1.0)
    assert math.isclose(d.radius, 2 * 0.25)                      # grid step 0.25: every point's nearest is 0.25 away
    q = np.array([[0.5, 0.5, 0.5, 0.5],                          # a training point
                  [0.62, -0.37, 0.88, 0.1],                      # between training points
                  [0.0, 0.0, 0.0, 0.0],                          # the middle of the hole (0.5 from the nearest)
                  [1.1, 0.0, 0.0, 0.0],                          # outside the box
                  [np.nan, 0.0, 0.0, 0.0]])
    assert d.contains(q).tolist() == [True, True, True, False, False]
    deep = _grid_with_hole()[np.any(np.abs(_grid_with_hole()) > 0.6, axis=1)]
    d2 = S.Domain.fit(deep)                                      # a wider hole: |x|_inf <= 0.6 empty
    assert not d2.contains([[0.0, 0.0, 0.0, 0.0]])[0]            # 0.75 from the nearest example > 0.5
    assert d2.contains([[0.75, 0.0, 0.0, 0.0]])[0]


def test_lens_for_matches_the_data_draw():
    """The fallback draws a parameter set's lens as the training data do."""
    rng = np.random.Generator(np.random.PCG64(5))
    lens, hx, hy = S.lens_for(0.5, 0.3, 0.6, 10.0, rng)
    kc, g1, g2, x, y, m = lens
    assert math.isclose(kc, 0.5 - 0.3) and g1 == 0.3 and g2 == 0.0
    assert math.isclose(hx, 5.0 / abs(1 - 0.5 - 0.3)) and math.isclose(hy, 5.0 / abs(1 - 0.5 + 0.3))
    r = 1.2 * math.hypot(hx, hy)
    assert len(x) == round(0.3 * r * r / S.W.salpeter_mean())
    assert np.all(np.hypot(x, y) <= math.sqrt(m.sum() / 0.3) * (1 + 1e-12))
    for bad in ((1.2, 0.2, 0.5), (0.5, 0.5, 0.5), (float("nan"), 0.1, 0.5), (0.5, 0.1, 1.5), (-0.1, 0.1, 0.5)):
        try:
            S.lens_for(*bad, 10.0, rng)
        except ValueError:
            continue
        raise AssertionError(f"no error for {bad}")
