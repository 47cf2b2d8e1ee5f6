"""ctypes wrapper of the C oracle (Eq. 1-3 and Algorithm 1 of arXiv:1703.09707).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy; everything is FP64 on the CPU,
single-threaded.  The lens is given as kappa_c, (gamma1, gamma2) and the star
arrays x, y, m; the ray lattice as (x0, y0, dx, dy, nx, ny, i0, j0); the
source window as (X0, Y0, Px, Py, NX, NY).
"""
import ctypes
import os
import types

import numpy as np

from . import build as _build

_D = ctypes.c_double
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def load_library(path):
    """Load an oracle build (the default one, or a test's own variant)."""
    lib = ctypes.CDLL(path)
    head = [_D, _D, _D, _I64, _P, _P, _P, _D, _D, _D, _D]
    win = [_D, _D, _D, _D, _I64, _I64]
    lib.ora_shoot.argtypes = head + [_I64, _I64, _I64, _I64] + win + [_P, _P, _P]
    lib.ora_shoot.restype = None
    lib.ora_map.argtypes = head + [_I64, _I64, _I64, _I64] + win + [_P]
    lib.ora_map.restype = _I64
    lib.ora_shoot_list.argtypes = head + [_I64, _P, _P] + win + [_P, _P, _P]
    lib.ora_shoot_list.restype = None
    lib.ora_error_scale.argtypes = [_D, _D, _D, _I64, _P, _P, _P, _D, _D]
    lib.ora_error_scale.restype = _D
    lib.ora_error_scale_block.argtypes = head + [_I64, _I64, _I64, _I64, _P]
    lib.ora_error_scale_block.restype = None
    return lib


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build_oracle()
        _lib = load_library(_build.LIB)
    return _lib


def _stars(x, y, m):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    assert x.shape == y.shape == m.shape and x.ndim == 1
    return x, y, m


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def shoot(lens, rays, pix, lib=None):
    """Per-ray (beta_x, beta_y, bin) arrays of shape (ny, nx); bin is -1
    for rays dropped or outside the window."""
    kc, g1, g2, x, y, m = lens
    x, y, m = _stars(x, y, m)
    x0, y0, dx, dy, nx, ny, i0, j0 = rays
    X0, Y0, Px, Py, NX, NY = pix
    bx = np.empty((ny, nx), np.float64)
    by = np.empty((ny, nx), np.float64)
    b = np.empty((ny, nx), np.int64)
    (lib or _load()).ora_shoot(kc, g1, g2, len(x), _ptr(x), _ptr(y), _ptr(m),
                      x0, y0, dx, dy, nx, ny, i0, j0,
                      X0, Y0, Px, Py, NX, NY, _ptr(bx), _ptr(by), _ptr(b))
    return bx, by, b


def map_counts(lens, rays, pix, counts=None, lib=None):
    """Algorithm 1: accumulate one count per binned ray into counts (NY, NX)
    int32 (a new zero map when None).  Returns (counts, n_binned)."""
    kc, g1, g2, x, y, m = lens
    x, y, m = _stars(x, y, m)
    x0, y0, dx, dy, nx, ny, i0, j0 = rays
    X0, Y0, Px, Py, NX, NY = pix
    if counts is None:
        counts = np.zeros((NY, NX), np.int32)
    assert counts.dtype == np.int32 and counts.shape == (NY, NX) and counts.flags.c_contiguous
    n = (lib or _load()).ora_map(kc, g1, g2, len(x), _ptr(x), _ptr(y), _ptr(m),
                        x0, y0, dx, dy, nx, ny, i0, j0,
                        X0, Y0, Px, Py, NX, NY, _ptr(counts))
    return counts, int(n)


def shoot_list(lens, rays, pix, ii, jj, lib=None):
    """Source angles and bins of the rays at global lattice indices (ii, jj)
    of the lattice (x0, y0, dx, dy); the rays' own nx, ny, i0, j0 are ignored."""
    kc, g1, g2, x, y, m = lens
    x, y, m = _stars(x, y, m)
    x0, y0, dx, dy = rays[:4]
    X0, Y0, Px, Py, NX, NY = pix
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    n = len(ii)
    bx = np.empty(n, np.float64)
    by = np.empty(n, np.float64)
    b = np.empty(n, np.int64)
    (lib or _load()).ora_shoot_list(kc, g1, g2, len(x), _ptr(x), _ptr(y), _ptr(m),
                           x0, y0, dx, dy, n, _ptr(ii), _ptr(jj),
                           X0, Y0, Px, Py, NX, NY, _ptr(bx), _ptr(by), _ptr(b))
    return bx, by, b


def error_scale(lens, tx, ty, lib=None):
    """S = |theta|_inf + |K theta|_inf + sum_k m_k/r_k for each ray (tx, ty)."""
    kc, g1, g2, x, y, m = lens
    x, y, m = _stars(x, y, m)
    lib = lib or _load()
    tx = np.atleast_1d(np.asarray(tx, np.float64))
    ty = np.atleast_1d(np.asarray(ty, np.float64))
    return np.array([lib.ora_error_scale(kc, g1, g2, len(x), _ptr(x), _ptr(y), _ptr(m),
                                         float(a), float(b)) for a, b in zip(tx, ty)])


def error_scale_block(lens, rays, lib=None):
    """Error scale S of every ray of a lattice block, shape (ny, nx)."""
    kc, g1, g2, x, y, m = lens
    x, y, m = _stars(x, y, m)
    x0, y0, dx, dy, nx, ny, i0, j0 = rays
    out = np.empty((ny, nx), np.float64)
    (lib or _load()).ora_error_scale_block(kc, g1, g2, len(x), _ptr(x), _ptr(y), _ptr(m),
                                           x0, y0, dx, dy, nx, ny, i0, j0, _ptr(out))
    return out


def image_angles(rays):
    """Cell-centred image angles (theta_x of each column, theta_y of each row)
    of a lattice, computed with the same roundings as the C code."""
    x0, y0, dx, dy, nx, ny, i0, j0 = rays
    tx = x0 + ((np.arange(i0, i0 + nx, dtype=np.int64).astype(np.float64) + 0.5) * dx)
    ty = y0 + ((np.arange(j0, j0 + ny, dtype=np.int64).astype(np.float64) + 0.5) * dy)
    return tx, ty


def bound(path):
    """A namespace with this module's functions bound to the oracle build
    at path (used by the tests that plant mistakes in a copy of the oracle)."""
    lib = load_library(path)
    ns = types.SimpleNamespace()
    ns.shoot = lambda lens, rays, pix: shoot(lens, rays, pix, lib=lib)
    ns.map_counts = lambda lens, rays, pix, counts=None: map_counts(lens, rays, pix, counts, lib=lib)
    ns.shoot_list = lambda lens, rays, pix, ii, jj: shoot_list(lens, rays, pix, ii, jj, lib=lib)
    ns.error_scale = lambda lens, tx, ty: error_scale(lens, tx, ty, lib=lib)
    ns.image_angles = image_angles
    return ns
