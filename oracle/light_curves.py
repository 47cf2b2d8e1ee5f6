"""FP64 oracle of simulated light curves: TEST INFRASTRUCTURE ONLY.

A magnification map and a model of the source's size and brightness profile
give simulated microlensing light curves (arXiv:1703.09707, Sec. 1).  The
paper fixes neither the profile nor how the source crosses the map; the
readings written out here are:

Source map (the map seen by a source of finite size):
  * mu = counts * norm, norm = (dx*dy)/(Px*Py) (ray counts are proportional
    to magnification, Sec. 1).
  * Gaussian profile of width sigma: the separable convolution of the
    surrogate's oracle (taps at pixel offsets |k| <= ceil(3 sigma / P),
    normalised per axis, rows then columns).
  * Uniform disk of radius R: the pixels at offsets (k, l) with
    (k Px)^2 + (l Py)^2 <= R^2, evaluated in FP64 as written, each squared
    term a product of its own.  The source-map value is
    (norm * S) / n, S the integer sum of the counts over those pixels and n
    their number.  rx and ry are the largest |k| on row l = 0 and the
    largest |l| on column k = 0 for which the test holds.
  * Only pixels at least (rx, ry) from every edge are kept: the source map
    has (NX - 2 rx) x (NY - 2 ry) pixels; its pixel (i, j) is pixel
    (i + rx, j + ry) of the map.

Light curves (tracks across the source map):
  * The source map is a grid of pixels (x0, y0, px, py, nx, ny); its
    values sit at the pixel centres, so an angle x has the continuous
    centre index (x - x0) / px - 0.5.
  * A track is a straight segment from a = (xa, ya) to b = (xb, yb) in
    source-plane angles, sampled at n points spaced evenly from a to b,
    computed in centre-index space with each reciprocal rounded once:
        ipx = 1 / px, inv = 1 / (n - 1) (inv = 0 when n == 1)
        u_a = (xa - x0) * ipx - 0.5,  du = ((xb - xa) * ipx) * inv
        u_k = u_a + du * k             (likewise v_k with y, py)
  * A sample with 0 <= u <= nx - 1 and 0 <= v <= ny - 1 takes the bilinear
    interpolation of its four surrounding centres, i = min(floor(u), nx - 2),
    fx = u - i (likewise j, fy):
        r0 = m[j][i] + fx (m[j][i+1] - m[j][i])
        r1 = m[j+1][i] + fx (m[j+1][i+1] - m[j+1][i])
        value = r0 + fy (r1 - r0)
    and any other sample (a NaN coordinate included) is NaN.  A single
    point x is evaluated at u = (x - x0) * ipx - 0.5.  The grid needs
    nx, ny >= 2.
"""
import math

import numpy as np

from oracle import surrogate as S

GAUSSIAN = 0
DISK = 1


# ----------------------------------------------------------------- source profiles
def disk_in(k, l, px, py, radius):
    """The disk test for the pixel offset (k, l), exactly as stated above."""
    a = float(k) * px
    b = float(l) * py
    return a * a + b * b <= radius * radius


def disk_radii(radius, px, py):
    """(rx, ry): the disk's half-widths along row 0 and column 0."""
    rx = 0
    while disk_in(rx + 1, 0, px, py, radius):
        rx += 1
    ry = 0
    while disk_in(0, ry + 1, px, py, radius):
        ry += 1
    return rx, ry


def disk_offsets(radius, px, py):
    """All (k, l) offsets inside the disk, l outer and k inner, increasing."""
    rx, ry = disk_radii(radius, px, py)
    return [(k, l) for l in range(-ry, ry + 1) for k in range(-rx, rx + 1)
            if disk_in(k, l, px, py, radius)]


def source_radii(profile, size, px, py):
    if profile == GAUSSIAN:
        return int(math.ceil(3.0 * size / px)), int(math.ceil(3.0 * size / py))
    if profile == DISK:
        return disk_radii(size, px, py)
    raise ValueError("unknown profile")


def source_map(counts, norm, profile, size, px, py):
    """The map seen by the source: FP64 array (NY - 2 ry, NX - 2 rx)."""
    counts = np.asarray(counts)
    ny, nx = counts.shape
    rx, ry = source_radii(profile, size, px, py)
    wx, wy = nx - 2 * rx, ny - 2 * ry
    if wx <= 0 or wy <= 0:
        raise ValueError("source larger than the map")
    if profile == GAUSSIAN:
        return S.smooth(np.asarray(counts, np.float64) * norm, size, px, py)
    total = np.zeros((wy, wx), np.int64)
    offs = disk_offsets(size, px, py)
    c = counts.astype(np.int64)
    for k, l in offs:
        total += c[ry + l:ry + l + wy, rx + k:rx + k + wx]
    return (norm * total.astype(np.float64)) / float(len(offs))


# ----------------------------------------------------------------- light curves
def sample_indices(grid, xa, ya, xb, yb, n):
    """Continuous centre indices (u, v), each (n_tracks, n), of the samples
    of straight tracks."""
    x0, y0, px, py = grid[:4]
    ipx = 1.0 / px
    ipy = 1.0 / py
    inv = 1.0 / float(n - 1) if n > 1 else 0.0
    xa, ya, xb, yb = (np.asarray(v, np.float64)[:, None] for v in (xa, ya, xb, yb))
    k = np.arange(n, dtype=np.float64)[None, :]
    ua = (xa - x0) * ipx - 0.5
    va = (ya - y0) * ipy - 0.5
    du = ((xb - xa) * ipx) * inv
    dv = ((yb - ya) * ipy) * inv
    return ua + du * k, va + dv * k


def interpolate_indices(mu_s, u, v):
    """Bilinear value of the source map at continuous centre indices
    (u, v); NaN outside the hull of the centres."""
    mu_s = np.asarray(mu_s, np.float64)
    ny, nx = mu_s.shape
    assert nx >= 2 and ny >= 2
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    out = np.full(u.shape, np.nan)
    for idx in np.ndindex(u.shape):
        uu, vv = float(u[idx]), float(v[idx])
        if not (0.0 <= uu <= nx - 1 and 0.0 <= vv <= ny - 1):
            continue
        i = min(int(math.floor(uu)), nx - 2)
        j = min(int(math.floor(vv)), ny - 2)
        fx = uu - i
        fy = vv - j
        r0 = mu_s[j, i] + fx * (mu_s[j, i + 1] - mu_s[j, i])
        r1 = mu_s[j + 1, i] + fx * (mu_s[j + 1, i + 1] - mu_s[j + 1, i])
        out[idx] = r0 + fy * (r1 - r0)
    return out


def interpolate(mu_s, grid, x, y):
    """Bilinear value of the source map at the angles (x, y); NaN outside."""
    x0, y0, px, py, nx, ny = grid
    assert np.shape(mu_s) == (ny, nx)
    u = (np.asarray(x, np.float64) - x0) * (1.0 / px) - 0.5
    v = (np.asarray(y, np.float64) - y0) * (1.0 / py) - 0.5
    return interpolate_indices(mu_s, u, v)


def light_curves(mu_s, grid, xa, ya, xb, yb, n_samples):
    """Light curves (n_tracks, n_samples) of straight tracks across mu_s."""
    assert np.shape(mu_s) == (grid[5], grid[4])
    u, v = sample_indices(grid, xa, ya, xb, yb, n_samples)
    return interpolate_indices(mu_s, u, v)


def source_grid(pix, profile, size):
    """The source map's own pixel grid (x0, y0, px, py, nx, ny), given the
    map's window pix = (X0, Y0, Px, Py, NX, NY)."""
    X0, Y0, Px, Py, NX, NY = pix
    rx, ry = source_radii(profile, size, Px, Py)
    return (X0 + rx * Px, Y0 + ry * Py, Px, Py, NX - 2 * rx, NY - 2 * ry)
