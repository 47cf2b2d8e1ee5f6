"""Exact rational ray shooting for tiny inputs: TEST INFRASTRUCTURE ONLY.

Every FP64 input is an exact binary rational, so Eq. (1) of arXiv:1703.09707
(Sec. 1) evaluated with Python's Fraction gives the exact source angle of
each ray, and the floor of (beta - X0)/Px gives its exact pixel.  This pins
the FP64 oracle: the two may differ only on rays whose exact pixel
coordinate lies within rounding of a pixel edge.

The image angle is the lattice point theta = origin + (idx + 1/2) * step
evaluated exactly; on a dyadic lattice that equals the FP64 value.
A ray exactly on a star has no finite source angle and is dropped (None).
"""
from fractions import Fraction as F
import math


def exact_beta(kappa_c, gamma1, gamma2, xs, ys, ms, tx, ty):
    """Exact (beta_x, beta_y) of Eq. (1) at image angle (tx, ty), or None
    when the ray sits exactly on a star."""
    tx, ty = F(tx), F(ty)
    kc, g1, g2 = F(kappa_c), F(gamma1), F(gamma2)
    # Eq. (1): beta = [[1-kc-g1, -g2], [-g2, 1-kc+g1]] theta - sum_k m_k (theta - theta_k)/|theta - theta_k|^2
    bx = (1 - kc - g1) * tx - g2 * ty
    by = -g2 * tx + (1 - kc + g1) * ty
    for x, y, m in zip(xs, ys, ms):
        ex, ey = tx - F(x), ty - F(y)
        r2 = ex * ex + ey * ey
        if r2 == 0:
            return None
        bx -= F(m) * ex / r2
        by -= F(m) * ey / r2
    return bx, by


def exact_pixel(beta, X0, Y0, Px, Py, NX, NY):
    """(linear index or -1, distance of the pixel coordinate to the nearest
    pixel edge as a float) for an exact source angle."""
    if beta is None:
        return -1, math.inf
    u = (beta[0] - F(X0)) / F(Px)
    v = (beta[1] - F(Y0)) / F(Py)
    du = min(u - math.floor(u), math.floor(u) + 1 - u)
    dv = min(v - math.floor(v), math.floor(v) + 1 - v)
    edge = float(min(du, dv, abs(u), abs(v), abs(u - NX), abs(v - NY)))
    if not (0 <= u < NX and 0 <= v < NY):
        return -1, edge
    return int(math.floor(v)) * NX + int(math.floor(u)), edge


def exact_shoot(lens, rays, pix):
    """Exact per-ray (beta or None, bin, edge distance), j-major lists."""
    kc, g1, g2, xs, ys, ms = lens
    x0, y0, dx, dy, nx, ny, i0, j0 = rays
    out = []
    for j in range(ny):
        ty = F(y0) + (F(j0 + j) + F(1, 2)) * F(dy)
        for i in range(nx):
            tx = F(x0) + (F(i0 + i) + F(1, 2)) * F(dx)
            b = exact_beta(kc, g1, g2, xs, ys, ms, tx, ty)
            p, e = exact_pixel(b, *pix)
            out.append((b, p, e))
    return out
