"""Seeded synthetic workloads: star fields, ray lattices and source windows.

This module generates inputs only.  It holds none of the ray-shooting
arithmetic, so that the GPU library and the independent CPU oracle both take
their inputs from here and share nothing else.

Conventions (arXiv:1703.09707, Sec. 1 and Sec. 3):
  * angles are in units of the Einstein angle of the mass unit and masses in
    that unit (Eq. 4 and the text after it);
  * stars are uniform in a disk centred on the origin (the paper only says
    "random star field"), with the disk radius chosen from the realised masses
    so that the stellar convergence kappa_star is exact.  In the units of
    Eq. (1) a star of mass m has Einstein radius sqrt(m), i.e. it carries a
    convergence integral of pi m, so a disk of radius R holding masses m_k has
    kappa_star = sum m_k / R^2 and R = sqrt(sum m / kappa_star);
  * the ray lattice covers the axis-aligned preimage, under the mean lens
    matrix A = [[1-k-g1, -g2], [-g2, 1-k+g1]] with k = kappa_c + kappa_star,
    of the source window (the paper's "lens window", Sec. 1);
  * masses are equal, Salpeter (dN/dm ~ m^-2.35 on [0.1, 1]) or log-uniform
    (Sec. 3 uses log-uniform on [0.01, 1.6]).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 170309707
SALPETER_SLOPE = 2.35


@dataclasses.dataclass
class Lens:
    """Macro parameters and star field of Eq. (1): kappa_c, (gamma1, gamma2)
    and stars at (x, y) with masses m (FP64 arrays, SoA)."""
    kappa_c: float
    gamma1: float
    gamma2: float
    x: np.ndarray
    y: np.ndarray
    m: np.ndarray
    kappa_star: float = 0.0

    @property
    def n_stars(self) -> int:
        return int(self.x.shape[0])

    def as_tuple(self):
        return (self.kappa_c, self.gamma1, self.gamma2, self.x, self.y, self.m)


@dataclasses.dataclass
class RayGrid:
    """Lattice of image angles: ray (i, j) of this block has global indices
    (i0 + i, j0 + j) and theta = (x0 + (i0+i+1/2) dx, y0 + (j0+j+1/2) dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int
    i0: int = 0
    j0: int = 0

    @property
    def n_rays(self) -> int:
        return self.nx * self.ny

    def as_tuple(self):
        return (self.x0, self.y0, self.dx, self.dy, self.nx, self.ny, self.i0, self.j0)

    def block(self, i0: int, j0: int, nx: int, ny: int) -> "RayGrid":
        """Sub-block of this lattice with the same origin and spacing."""
        return RayGrid(self.x0, self.y0, self.dx, self.dy, nx, ny,
                       self.i0 + i0, self.j0 + j0)


@dataclasses.dataclass
class PixelGrid:
    """Source window: pixel (is, js) = [X0 + is Px, X0 + (is+1) Px) x
    [Y0 + js Py, Y0 + (js+1) Py); map element js*NX + is."""
    X0: float
    Y0: float
    Px: float
    Py: float
    NX: int
    NY: int

    def as_tuple(self):
        return (self.X0, self.Y0, self.Px, self.Py, self.NX, self.NY)


@dataclasses.dataclass
class Workload:
    name: str
    lens: Lens
    rays: RayGrid
    pix: PixelGrid
    seed: int

    @property
    def interactions(self) -> int:
        return self.rays.n_rays * self.lens.n_stars


# ---------------------------------------------------------------- masses
def equal_masses(n: int, m: float = 1.0) -> np.ndarray:
    return np.full(n, m, np.float64)


def salpeter_masses(n: int, rng: np.random.Generator, lo: float = 0.1,
                    hi: float = 1.0, slope: float = SALPETER_SLOPE) -> np.ndarray:
    """Inverse-CDF draw from dN/dm ~ m^-slope on [lo, hi]."""
    a = 1.0 - slope
    u = rng.random(n)
    return (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)


def salpeter_mean(lo: float = 0.1, hi: float = 1.0, slope: float = SALPETER_SLOPE) -> float:
    a1, a2 = 2.0 - slope, 1.0 - slope
    return ((hi ** a1 - lo ** a1) / a1) / ((hi ** a2 - lo ** a2) / a2)


def log_uniform_masses(n: int, rng: np.random.Generator, lo: float = 0.01,
                       hi: float = 1.6) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


# ---------------------------------------------------------------- positions
def disk_positions(n: int, radius: float, rng: np.random.Generator):
    """Uniform in a disk: r = R sqrt(u1), phi = 2 pi u2."""
    u1 = rng.random(n)
    u2 = rng.random(n)
    r = radius * np.sqrt(u1)
    phi = 2.0 * math.pi * u2
    return r * np.cos(phi), r * np.sin(phi)


def star_field(masses: np.ndarray, kappa_star: float, rng: np.random.Generator):
    """Positions uniform in the disk whose mean stellar convergence is
    exactly kappa_star for these masses: kappa_star = sum m / R^2."""
    radius = math.sqrt(float(masses.sum()) / kappa_star)
    x, y = disk_positions(len(masses), radius, rng)
    return np.ascontiguousarray(x), np.ascontiguousarray(y), radius


# ---------------------------------------------------------------- geometry
def mean_lens_matrix(kappa: float, gamma1: float, gamma2: float) -> np.ndarray:
    return np.array([[1.0 - kappa - gamma1, -gamma2],
                     [-gamma2, 1.0 - kappa + gamma1]])


def preimage_half_widths(kappa: float, gamma1: float, gamma2: float,
                         half_x: float, half_y: float, margin: float = 1.0):
    """Half widths of the axis-aligned box around the preimage, under the
    mean lens matrix, of the window [-half_x, half_x] x [-half_y, half_y]."""
    ainv = np.linalg.inv(mean_lens_matrix(kappa, gamma1, gamma2))
    corners = np.array([[sx * half_x, sy * half_y] for sx in (-1, 1) for sy in (-1, 1)])
    pre = corners @ ainv.T
    return margin * float(np.abs(pre[:, 0]).max()), margin * float(np.abs(pre[:, 1]).max())


def centred_window(width: float, npix: int) -> PixelGrid:
    p = width / npix
    return PixelGrid(-width / 2, -width / 2, p, p, npix, npix)


def centred_rays(hx: float, hy: float, nx: int, ny: int) -> RayGrid:
    return RayGrid(-hx, -hy, 2 * hx / nx, 2 * hy / ny, nx, ny)


# ---------------------------------------------------------------- configs
def plain_fp64_small(seed: int = BASE_SEED) -> Workload:
    """100 unit-mass stars with kappa_star = 0.4, kappa_c = 0, gamma = (0.4, 0);
    1000 x 1000 rays; 256 x 256 map over 10 x 10 Einstein angles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, kc, g1, g2 = 0.4, 0.0, 0.4, 0.0
    m = equal_masses(100)
    x, y, _ = star_field(m, ks, rng)
    pix = centred_window(10.0, 256)
    hx, hy = preimage_half_widths(kc + ks, g1, g2, 5.0, 5.0)
    rays = centred_rays(hx, hy, 1000, 1000)
    return Workload("plain-fp64-small: N*=100 m=1, 1000^2 rays, 256^2 map",
                    Lens(kc, g1, g2, x, y, m, ks), rays, pix, seed)


def plain_fp64_large(seed: int = BASE_SEED + 1) -> Workload:
    """16384 Salpeter stars, kappa_star = 0.3, kappa_c = 0.15,
    gamma = (0.35, 0.1); 8192 x 8192 rays; 1024 x 1024 map over 20 x 20."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, kc, g1, g2 = 0.3, 0.15, 0.35, 0.1
    m = salpeter_masses(16384, rng)
    x, y, _ = star_field(m, ks, rng)
    pix = centred_window(20.0, 1024)
    hx, hy = preimage_half_widths(kc + ks, g1, g2, 10.0, 10.0)
    rays = centred_rays(hx, hy, 8192, 8192)
    return Workload("plain-fp64-large: N*=16384 Salpeter, 8192^2 rays, 1024^2 map",
                    Lens(kc, g1, g2, x, y, m, ks), rays, pix, seed)


def precision_study(seed: int = BASE_SEED + 2) -> Workload:
    """262144 Salpeter stars, kappa_star = 0.45, kappa_c = 0, gamma = (0.45, 0);
    16384 x 16384 rays over [-100, 100] x [-10, 10] (dyadic spacing);
    2048 x 2048 map over 20 x 20."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, kc, g1, g2 = 0.45, 0.0, 0.45, 0.0
    m = salpeter_masses(262144, rng)
    x, y, _ = star_field(m, ks, rng)
    pix = centred_window(20.0, 2048)
    hx, hy = preimage_half_widths(kc + ks, g1, g2, 10.0, 10.0)
    rays = centred_rays(hx, hy, 16384, 16384)
    return Workload("precision-study: N*=262144 Salpeter, 16384^2 rays, 2048^2 map",
                    Lens(kc, g1, g2, x, y, m, ks), rays, pix, seed)


def precision_subtile(w: Workload, n: int = 2048) -> RayGrid:
    """Central n x n block of a lattice."""
    return w.rays.block((w.rays.nx - n) // 2, (w.rays.ny - n) // 2, n, n)


def large_star_field(n_stars: int = 1 << 24, rays_per_side: int = 512, npix: int = 256,
                     seed: int = BASE_SEED + 5) -> Workload:
    """Many stars, few rays (the regime that Sec. 4 says needs the star sum
    split across threads): n_stars Salpeter stars with kappa_star = 0.45,
    kappa_c = 0, gamma = (0.3, 0); a rays_per_side^2 lattice over the
    preimage of a 2 x 2 window around the centre; npix^2 map."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, kc, g1, g2 = 0.45, 0.0, 0.3, 0.0
    m = salpeter_masses(n_stars, rng)
    x, y, _ = star_field(m, ks, rng)
    pix = centred_window(2.0, npix)
    hx, hy = preimage_half_widths(kc + ks, g1, g2, 1.0, 1.0)
    rays = centred_rays(hx, hy, rays_per_side, rays_per_side)
    return Workload(f"large-star-field: N*={n_stars} Salpeter, {rays_per_side}^2 rays, {npix}^2 map",
                    Lens(kc, g1, g2, x, y, m, ks), rays, pix, seed)


def draw_batch_params(rng: np.random.Generator, n_sets: int, n_lo: int = 500,
                      n_hi: int = 50000, window: float = 10.0):
    """Rejection draw of (kappa, gamma, kappa_star/kappa) with
    kappa ~ U[0.2, 0.8], gamma ~ U[0.1, 0.6] (gamma2 = 0), f ~ U[0.1, 1];
    the lens-window radius is 1.2 x the preimage box's half diagonal and
    N* = round(kappa_star R^2 / <m>) (the star count of convergence
    kappa_star in a disk of radius R) must lie in [n_lo, n_hi]."""
    mbar = salpeter_mean()
    out = []
    draws = 0
    while len(out) < n_sets:
        kappa = rng.uniform(0.2, 0.8)
        gamma = rng.uniform(0.1, 0.6)
        f = rng.uniform(0.1, 1.0)
        draws += 1
        det = (1 - kappa) ** 2 - gamma ** 2
        if abs(det) < 1e-3:
            continue
        hx, hy = preimage_half_widths(kappa, gamma, 0.0, window / 2, window / 2)
        radius = 1.2 * math.hypot(hx, hy)
        ks = f * kappa
        n = int(round(ks * radius ** 2 / mbar))
        if n_lo <= n <= n_hi:
            out.append(dict(kappa=kappa, gamma=gamma, f=f, kappa_star=ks,
                            kappa_c=kappa - ks, n_stars=n, hx=hx, hy=hy))
    return out, draws


def batch_workloads(n_sets: int = 64, rays_per_side: int = 4096, npix: int = 512,
                    window: float = 10.0, seed: int = BASE_SEED + 3,
                    n_lo: int = 500, n_hi: int = 50000) -> list[Workload]:
    """Parameter sets of uneven star counts, each with its own star field,
    ray lattice over its own preimage box and a 512^2 map over 10 x 10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params, _ = draw_batch_params(rng, n_sets, n_lo, n_hi, window)
    out = []
    for s, p in enumerate(params):
        srng = np.random.Generator(np.random.PCG64(seed + 1000 * 3 + s))
        m = salpeter_masses(p["n_stars"], srng)
        x, y, _ = star_field(m, p["kappa_star"], srng)
        rays = centred_rays(p["hx"], p["hy"], rays_per_side, rays_per_side)
        pix = centred_window(window, npix)
        lens = Lens(p["kappa_c"], p["gamma"], 0.0, x, y, m, p["kappa_star"])
        out.append(Workload(f"batch-set-{s}", lens, rays, pix, seed + 1000 * 3 + s))
    return out


def mean_magnification(kappa: float, gamma1: float, gamma2: float) -> float:
    """1 / |det A| for the mean lens matrix: the textbook mean magnification
    of a smooth sheet, also the large-field mean for a star field."""
    return 1.0 / abs((1.0 - kappa) ** 2 - gamma1 ** 2 - gamma2 ** 2)


# ----------------------------------------------------------------- light curves
def light_curve_tracks(grid, n_tracks: int, length: float, seed: int = BASE_SEED + 5):
    """Straight tracks of the given length across a source map's pixel grid
    grid = (x0, y0, px, py, nx, ny): centres uniform in the hull of the
    pixel centres shrunk by length / 2 on every side, directions uniform.
    Returns FP64 arrays (xa, ya, xb, yb)."""
    x0, y0, px, py, nx, ny = grid
    lo_x, hi_x = x0 + 0.5 * px + 0.5 * length, x0 + (nx - 0.5) * px - 0.5 * length
    lo_y, hi_y = y0 + 0.5 * py + 0.5 * length, y0 + (ny - 0.5) * py - 0.5 * length
    if not (lo_x < hi_x and lo_y < hi_y):
        raise ValueError("tracks longer than the map")
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(lo_x, hi_x, n_tracks)
    cy = rng.uniform(lo_y, hi_y, n_tracks)
    phi = rng.uniform(0.0, 2.0 * math.pi, n_tracks)
    hx, hy = 0.5 * length * np.cos(phi), 0.5 * length * np.sin(phi)
    return cx - hx, cy - hy, cx + hx, cy + hy


@dataclasses.dataclass
class LightCurveWorkload:
    """Light curves across the map of a ray-shooting workload."""
    name: str
    maps: Workload
    profile: str
    size: float
    n_tracks: int
    n_samples: int
    length: float


def light_curves_large() -> LightCurveWorkload:
    """The 1024^2 map of plain-fp64-large (20 x 20 Einstein angles), a
    Gaussian source of width 2 pixels, and 2^20 tracks of 2 Einstein angles
    sampled at 256 points (about 0.4 pixel apart)."""
    w = plain_fp64_large()
    return LightCurveWorkload("light-curves-large: 2^20 tracks x 256 samples on the 1024^2 map of "
                              "plain-fp64-large, Gaussian source of 2 pixels", w, "gaussian",
                              2.0 * w.pix.Px, 1 << 20, 256, 2.0)
