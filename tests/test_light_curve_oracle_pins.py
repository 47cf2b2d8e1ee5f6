"""Pins of the light-curve oracle against closed forms, exact counts and the
point-lens magnification.

Every pin_* function takes the oracle module as its argument so that
test_light_curve_mutants.py can run the same pins against copies of the
oracle with planted mistakes.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import light_curves as LC
from oracle import shooter as ora

# Lattice points (k, l) with k^2 + l^2 <= R^2 for R = 1..10 (Gauss's circle
# problem; OEIS A000328).
GAUSS_CIRCLE = [5, 13, 29, 49, 81, 113, 149, 197, 253, 317]


def _grid():
    # non-square pixels and map, so that a transposed index shows
    return (-1.25, 0.75, 0.125, 0.0625, 23, 17)


def _centres(grid):
    x0, y0, px, py, nx, ny = grid
    xc = np.array([float(Fraction(x0) + (i + Fraction(1, 2)) * Fraction(px)) for i in range(nx)])
    yc = np.array([float(Fraction(y0) + (j + Fraction(1, 2)) * Fraction(py)) for j in range(ny)])
    return xc, yc


def pin_linear_map_is_reproduced(L):
    """Bilinear interpolation reproduces a linear function exactly (up to
    rounding) anywhere in the hull of the pixel centres, the far edges
    included."""
    grid = _grid()
    xc, yc = _centres(grid)
    m = 2.0 + 3.0 * xc[None, :] + 5.0 * yc[:, None]
    # dyadic tracks sampled at 9 points (s = k/8 exact)
    xa = np.array([xc[0], xc[3] + 0.03125, xc[-1], xc[0]])
    ya = np.array([yc[0], yc[2], yc[-1], yc[-1]])
    xb = np.array([xc[-1], xc[10] - 0.0625, xc[0], xc[-1]])
    yb = np.array([yc[-1], yc[-4] + 0.015625, yc[0], yc[0]])
    got = L.light_curves(m, grid, xa, ya, xb, yb, 9)
    s = np.arange(9) / 8.0
    for t in range(4):
        x = np.array([float(Fraction(xa[t]) + (Fraction(xb[t]) - Fraction(xa[t])) * Fraction(k, 8))
                      for k in range(9)])
        y = np.array([float(Fraction(ya[t]) + (Fraction(yb[t]) - Fraction(ya[t])) * Fraction(k, 8))
                      for k in range(9)])
        want = 2.0 + 3.0 * x + 5.0 * y
        np.testing.assert_allclose(got[t], want, rtol=1e-13, atol=1e-13)
    assert s[-1] == 1.0


def pin_pixel_centres_are_exact(L):
    grid = _grid()
    xc, yc = _centres(grid)
    rng = np.random.default_rng(3)
    m = rng.uniform(0.1, 10.0, (grid[5], grid[4]))
    ii = rng.integers(0, grid[4], 40)
    jj = rng.integers(0, grid[5], 40)
    got = L.interpolate(m, grid, xc[ii], yc[jj])
    np.testing.assert_array_equal(got, m[jj, ii])


def pin_hull_and_nan(L):
    grid = _grid()
    x0, y0, px, py, nx, ny = grid
    xc, yc = _centres(grid)
    m = np.arange(nx * ny, dtype=np.float64).reshape(ny, nx)
    inside = L.interpolate(m, grid, np.array([xc[0], xc[-1], xc[-1]]), np.array([yc[0], yc[-1], yc[0]]))
    np.testing.assert_array_equal(inside, [m[0, 0], m[-1, -1], m[0, -1]])
    eps = 1e-9
    out = L.interpolate(m, grid, np.array([xc[0] - eps, xc[-1] + eps, xc[5], xc[5], np.nan, xc[2]]),
                        np.array([yc[3], yc[3], yc[0] - eps, yc[-1] + eps, yc[2], np.nan]))
    assert np.all(np.isnan(out))


def pin_sample_positions(L):
    """Samples sit at the centre indices of points spaced evenly from a to
    b (exact for dyadic tracks), and a single sample at a."""
    grid = _grid()
    x0, y0, px, py = grid[:4]
    xa, ya, xb, yb = [0.5, -1.0], [0.25, 2.0], [-1.5, 1.0], [1.25, 2.0]
    u, v = L.sample_indices(grid, np.array(xa), np.array(ya), np.array(xb), np.array(yb), 5)
    for t in range(2):
        for k in range(5):
            x = Fraction(xa[t]) + (Fraction(xb[t]) - Fraction(xa[t])) * Fraction(k, 4)
            y = Fraction(ya[t]) + (Fraction(yb[t]) - Fraction(ya[t])) * Fraction(k, 4)
            assert u[t, k] == float((x - Fraction(x0)) / Fraction(px) - Fraction(1, 2))
            assert v[t, k] == float((y - Fraction(y0)) / Fraction(py) - Fraction(1, 2))
    u, v = L.sample_indices(grid, np.array([0.5]), np.array([0.25]), np.array([9.0]), np.array([9.0]), 1)
    assert u.shape == (1, 1)
    assert u[0, 0] == float((Fraction(0.5) - Fraction(x0)) / Fraction(px) - Fraction(1, 2))
    assert v[0, 0] == float((Fraction(0.25) - Fraction(y0)) / Fraction(py) - Fraction(1, 2))
    # tracks of many samples end within rounding of b
    u, v = L.sample_indices(grid, np.array([-1.2]), np.array([0.8]), np.array([1.3]), np.array([1.7]), 1001)
    assert abs(u[0, -1] - ((1.3 - x0) / px - 0.5)) < 1e-12
    assert abs(v[0, -1] - ((1.7 - y0) / py - 0.5)) < 1e-12
    assert abs(u[0, 500] - ((0.05 - x0) / px - 0.5)) < 1e-12


def pin_disk_offsets(L):
    """The disk's pixel set: Gauss's circle counts on unit pixels, and the
    exact lattice set on dyadic non-square pixels."""
    for r, n in enumerate(GAUSS_CIRCLE, start=1):
        assert len(L.disk_offsets(float(r), 1.0, 1.0)) == n, r
        assert L.disk_radii(float(r), 1.0, 1.0) == (r, r)
    px, py, R = 0.5, 0.25, 1.375
    want = {(k, l) for k in range(-10, 11) for l in range(-10, 11)
            if (Fraction(k) * Fraction(px)) ** 2 + (Fraction(l) * Fraction(py)) ** 2 <= Fraction(R) ** 2}
    got = L.disk_offsets(R, px, py)
    assert set(got) == want and len(got) == len(want)
    assert L.disk_radii(R, px, py) == (2, 5)
    assert L.source_radii(L.DISK, R, px, py) == (2, 5)
    assert L.source_radii(L.GAUSSIAN, 0.125, 0.03125, 0.0625) == (12, 6)
    assert L.source_radii(L.GAUSSIAN, 0.05, 0.03125, 0.0625) == (5, 3)


def pin_disk_source_map(L):
    """A single counted pixel spreads over the disk's pixels with weight
    norm/n; a constant map stays constant; a linear map stays linear."""
    px, py, R, norm = 0.5, 0.25, 1.375, 0.75
    offs = {(k, l) for k in range(-10, 11) for l in range(-10, 11)
            if (Fraction(k) * Fraction(px)) ** 2 + (Fraction(l) * Fraction(py)) ** 2 <= Fraction(R) ** 2}
    rx, ry = 2, 5
    NY, NX = 20, 16
    c = np.zeros((NY, NX), np.int32)
    c[9, 7] = 1
    got = L.source_map(c, norm, L.DISK, R, px, py)
    assert got.shape == (NY - 2 * ry, NX - 2 * rx)
    want = np.zeros_like(got)
    for j in range(got.shape[0]):
        for i in range(got.shape[1]):
            if (7 - (i + rx), 9 - (j + ry)) in offs:
                want[j, i] = norm / len(offs)
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)
    got = L.source_map(np.full((NY, NX), 7, np.int32), norm, L.DISK, R, px, py)
    np.testing.assert_array_equal(got, 7 * norm)
    jj, ii = np.mgrid[0:NY, 0:NX]
    lin = (3 + 2 * ii + 5 * jj).astype(np.int32)
    got = L.source_map(lin, norm, L.DISK, R, px, py)
    np.testing.assert_allclose(got, norm * lin[ry:NY - ry, rx:NX - rx], rtol=1e-15)


def pin_gaussian_source_map(L):
    norm, sigma, px, py = 0.5, 0.05, 0.03125, 0.0625
    rx, ry = 5, 3
    got = L.source_map(np.full((20, 30), 4, np.int32), norm, L.GAUSSIAN, sigma, px, py)
    assert got.shape == (20 - 2 * ry, 30 - 2 * rx)
    np.testing.assert_allclose(got, 2.0, rtol=1e-14)
    jj, ii = np.mgrid[0:20, 0:30]
    lin = (3 + 2 * ii + 5 * jj).astype(np.int32)
    got = L.source_map(lin, norm, L.GAUSSIAN, sigma, px, py)
    np.testing.assert_allclose(got, norm * lin[ry:20 - ry, rx:30 - rx], rtol=1e-13)


def pin_source_grid_places_values(L):
    """The source map's grid puts each value at its pixel's centre: for a
    linear count map, interpolating the source map at an angle gives the
    linear function of that angle."""
    pix = (-1.0, 0.5, 0.125, 0.0625, 40, 36)
    X0, Y0, Px, Py, NX, NY = pix
    jj, ii = np.mgrid[0:NY, 0:NX]
    lin = (1000 + 2 * ii + 5 * jj).astype(np.int32)
    for prof, size in ((L.GAUSSIAN, 0.1), (L.DISK, 0.3)):
        grid = L.source_grid(pix, prof, size)
        mu = L.source_map(lin, 1.0, prof, size, Px, Py)
        assert mu.shape == (grid[5], grid[4])
        x = np.array([-0.4, 0.9, 2.0])
        y = np.array([1.2, 1.7, 2.0])
        got = L.interpolate(mu, grid, x, y)
        want = 1000 + 2 * ((x - X0) / Px - 0.5) + 5 * ((y - Y0) / Py - 0.5)
        np.testing.assert_allclose(got, want, rtol=1e-12)


PINS = [pin_linear_map_is_reproduced, pin_pixel_centres_are_exact, pin_hull_and_nan, pin_sample_positions,
        pin_disk_offsets, pin_disk_source_map, pin_gaussian_source_map, pin_source_grid_places_values]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(LC)


# ----------------------------------------------------------------- point lens
def _point_lens_mu(u):
    """Point-source magnification of one unit-mass point lens."""
    return (u * u + 2.0) / (u * np.sqrt(u * u + 4.0))


@pytest.fixture(scope="module")
def point_lens_map(oracle_lib):
    """One unit-mass star at the origin, no smooth matter or shear: a
    128^2 map of [-2, 2]^2 from 8192^2 rays over [-4, 4]^2."""
    lens = (0.0, 0.0, 0.0, [0.0], [0.0], [1.0])
    rays = (-4.0, -4.0, 8 / 8192, 8 / 8192, 8192, 8192, 0, 0)
    pix = (-2.0, -2.0, 4 / 128, 4 / 128, 128, 128)
    counts, _ = ora.map_counts(lens, rays, pix)
    norm = (rays[2] * rays[3]) / (pix[2] * pix[3])
    return counts, norm, pix


def test_point_lens_disk_source_at_the_lens(point_lens_map):
    """A uniform disk of radius rho centred on a point lens is magnified by
    sqrt(1 + 4 / rho^2) (finite-source point lens)."""
    counts, norm, pix = point_lens_map
    for rho in (0.25, 0.5):
        mu = LC.source_map(counts, norm, LC.DISK, rho, pix[2], pix[3])
        grid = LC.source_grid(pix, LC.DISK, rho)
        # the lens sits on a pixel corner: average the four values around it
        eps = 0.25 * pix[2]
        got = LC.interpolate(mu, grid, np.array([eps, -eps, eps, -eps]), np.array([eps, eps, -eps, -eps]))
        want = math.sqrt(1.0 + 4.0 / (rho * rho))
        assert abs(got.mean() / want - 1) < 0.015, (rho, got, want)


def test_point_lens_gaussian_light_curve(point_lens_map):
    """A Gaussian source crossing a point lens at impact parameter 0.6: the
    light curve follows the point-source magnification averaged over the
    source profile (2D quadrature), to the ray-counting error (a star 10%
    too heavy moves the curve by 2-4%)."""
    counts, norm, pix = point_lens_map
    sigma = 0.1
    mu = LC.source_map(counts, norm, LC.GAUSSIAN, sigma, pix[2], pix[3])
    grid = LC.source_grid(pix, LC.GAUSSIAN, sigma)
    lc = LC.light_curves(mu, grid, np.array([-1.2]), np.array([0.6]), np.array([1.2]), np.array([0.6]), 13)[0]
    # Gauss-Hermite product rule for the weight exp(-a^2/2) exp(-b^2/2)
    a, w = np.polynomial.hermite_e.hermegauss(32)
    A, B = np.meshgrid(a, a)
    W2 = np.outer(w, w) / (2 * math.pi)
    xs = np.linspace(-1.2, 1.2, 13)
    for x, got in zip(xs, lc):
        want = float((W2 * _point_lens_mu(np.hypot(x + sigma * A, 0.6 + sigma * B))).sum())
        assert abs(got / want - 1) < 3e-3, (x, got, want)
