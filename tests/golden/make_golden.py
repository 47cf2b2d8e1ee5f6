"""Write tests/golden/exact_tiny.json from the exact-rational oracle only.

The case: 5 stars (one placed exactly on a lattice point, so that ray is
dropped), smooth matter and shear, a 24 x 20 dyadic ray lattice and a
16 x 12 source window.  Stored: the inputs, the exact bin of every ray, the
distance of its exact pixel coordinate to the nearest edge, and the exact
map.  Lens equation: arXiv:1703.09707, Sec. 1, Eq. (1); steps: Algorithm 1.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import exact  # noqa: E402


def main():
    rng = np.random.default_rng(1703)
    xs = list(rng.uniform(-1.5, 1.5, 4)) + [0.421875]     # last star on lattice point (i=12, j=9)
    ys = list(rng.uniform(-1.5, 1.5, 4)) + [-0.09375]
    ms = list(rng.uniform(0.1, 0.9, 5))
    lens = (0.125, 0.1875, -0.0625, xs, ys, ms)
    rays = (-3.09375, -2.46875, 0.28125, 0.25, 24, 20, 0, 0)
    pix = (-2.0, -1.5, 0.25, 0.25, 16, 12)
    res = exact.exact_shoot(lens, rays, pix)
    counts = np.zeros(pix[5] * pix[4], np.int64)
    for _, p, _ in res:
        if p >= 0:
            counts[p] += 1
    out = {
        "source": "exact rational evaluation of Eq. (1) and Algorithm 1 of arXiv:1703.09707 "
                  "(oracle/exact.py); written by tests/golden/make_golden.py",
        "lens": {"kappa_c": lens[0], "gamma1": lens[1], "gamma2": lens[2],
                 "x": [float(v) for v in xs], "y": [float(v) for v in ys], "m": [float(v) for v in ms]},
        "rays": dict(zip(["x0", "y0", "dx", "dy", "nx", "ny", "i0", "j0"], rays)),
        "pix": dict(zip(["X0", "Y0", "Px", "Py", "NX", "NY"], pix)),
        "bins": [p for _, p, _ in res],
        "edge_distance": [min(e, 1.0) for _, _, e in res],
        "beta_x": [float(b[0]) if b is not None else None for b, _, _ in res],
        "beta_y": [float(b[1]) if b is not None else None for b, _, _ in res],
        "counts": counts.tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_tiny.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(path, "binned", int(counts.sum()), "dropped", sum(b is None for b, _, _ in res))


if __name__ == "__main__":
    main()
