"""Python binding of libraysh (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; torch is
used here only to allocate device memory and to name the HIP stream.  The
functions mirror the C ABI of include/raysh.h: ``Context`` wraps
raysh_init/raysh_free, ``Context.shoot`` raysh_shoot, ``Context.map``
raysh_map and ``map_batch`` raysh_map_batch.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libraysh.so")

FP64 = 0
FP32_BULK = 1
FP64_EXPANSION = 2
CELL_MODES = {"auto": 0, "always": 1, "never": 2}   # RAYSH_CELLS_*
PRECISIONS = {"fp64": FP64, "fp32_bulk": FP32_BULK, "fp64_expansion": FP64_EXPANSION,
              FP64: FP64, FP32_BULK: FP32_BULK, FP64_EXPANSION: FP64_EXPANSION}

SOURCE_GAUSSIAN = 0
SOURCE_DISK = 1
PROFILES = {"gaussian": SOURCE_GAUSSIAN, "disk": SOURCE_DISK,
            SOURCE_GAUSSIAN: SOURCE_GAUSSIAN, SOURCE_DISK: SOURCE_DISK}

OK, EINVAL, EOVERFLOW, ENOMEM, EDEVICE = 0, 1, 2, 3, 4
_CODES = {EINVAL: "EINVAL", EOVERFLOW: "EOVERFLOW", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE"}

EXPORTS = ("raysh_init", "raysh_set_stream", "raysh_n_stars", "raysh_set_tile", "raysh_set_star_split",
           "raysh_set_expansion", "raysh_set_expansion_block", "raysh_set_expansion_cells",
           "raysh_expansion_order",
           "raysh_list_tiles",
           "raysh_get_tile", "raysh_autotune", "raysh_autotune_batch", "raysh_shoot", "raysh_map", "raysh_map_split_noalloc",
           "raysh_map_batch",
           "raysh_histogram_workspace", "raysh_log_mag_histogram",
           "raysh_source_map_shape", "raysh_source_map_workspace", "raysh_source_map", "raysh_light_curves",
           "raysh_track_order_workspace", "raysh_track_order", "raysh_fma_probe", "raysh_set_lens",
           "raysh_mlp_create",
           "raysh_mlp_n_params", "raysh_mlp_get_params", "raysh_mlp_forward", "raysh_mlp_gradient",
           "raysh_mlp_adam_step", "raysh_mlp_train_step", "raysh_mlp_sync", "raysh_mlp_free",
           "raysh_sync", "raysh_free", "raysh_last_error")


class RayshError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Lens(ctypes.Structure):
    _fields_ = [("kappa_c", ctypes.c_double), ("gamma1", ctypes.c_double),
                ("gamma2", ctypes.c_double), ("n_stars", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("m", ctypes.c_void_p)]


class Rays(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("i0", ctypes.c_int64), ("j0", ctypes.c_int64)]


class Pixels(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("px", ctypes.c_double), ("py", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


_lib = None


def load():
    """Load libraysh.so; raises if it has not been built.

    torch is imported first: its wheel carries its own HIP runtime, and a
    process must use one HIP runtime only, so libraysh binds to the one torch
    has loaded instead of loading a second copy from the system."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see above)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1703_09707_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.raysh_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Lens), I, P]
    lib.raysh_set_stream.argtypes = [P, P]
    lib.raysh_n_stars.argtypes = [P]
    lib.raysh_n_stars.restype = ctypes.c_int64
    lib.raysh_set_tile.argtypes = [P, I, I, I, I, I]
    lib.raysh_get_tile.argtypes = [P, I] + [ctypes.POINTER(I)] * 4
    lib.raysh_set_expansion.argtypes = [P, ctypes.c_double]
    lib.raysh_set_expansion.restype = I
    lib.raysh_set_expansion_block.argtypes = [P, I]
    lib.raysh_set_expansion_block.restype = I
    lib.raysh_set_expansion_cells.argtypes = [P, I]
    lib.raysh_set_expansion_cells.restype = I
    lib.raysh_expansion_order.argtypes = []
    lib.raysh_expansion_order.restype = I
    lib.raysh_set_star_split.argtypes = [P, I]
    lib.raysh_set_star_split.restype = I
    lib.raysh_list_tiles.argtypes = [I, ctypes.POINTER(ctypes.c_int32), I]
    lib.raysh_list_tiles.restype = I
    lib.raysh_histogram_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.raysh_histogram_workspace.restype = ctypes.c_size_t
    D = ctypes.c_double
    lib.raysh_log_mag_histogram.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, D, D, D, D,
                                            ctypes.c_int32, D, D, P, ctypes.c_size_t, P, P, P]
    lib.raysh_log_mag_histogram.restype = I
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.raysh_source_map_shape.argtypes = [ctypes.c_int32, ctypes.c_int32, I, D, D, D, i32p, i32p]
    lib.raysh_source_map_shape.restype = I
    lib.raysh_source_map_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.raysh_source_map_workspace.restype = ctypes.c_size_t
    lib.raysh_source_map.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, I, D, D, D, P, ctypes.c_size_t, P, P]
    lib.raysh_source_map.restype = I
    lib.raysh_light_curves.argtypes = [P, ctypes.POINTER(Pixels), ctypes.c_int64, ctypes.c_int32,
                                       P, P, P, P, P, P, P, P]
    lib.raysh_light_curves.restype = I
    lib.raysh_track_order_workspace.argtypes = [ctypes.POINTER(Pixels)]
    lib.raysh_track_order_workspace.restype = ctypes.c_size_t
    lib.raysh_track_order.argtypes = [ctypes.POINTER(Pixels), ctypes.c_int64, P, P, P, P, P, ctypes.c_size_t, P, P,
                                      P]
    lib.raysh_track_order.restype = I
    lib.raysh_set_lens.argtypes = [P, ctypes.POINTER(Lens)]
    lib.raysh_set_lens.restype = I
    lib.raysh_fma_probe.argtypes = [I, ctypes.c_int64, ctypes.c_int32, P, P]
    lib.raysh_fma_probe.restype = I
    F = ctypes.c_float
    lib.raysh_mlp_create.argtypes = [ctypes.POINTER(P), I, P, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, P]
    lib.raysh_mlp_n_params.argtypes = [P]
    lib.raysh_mlp_n_params.restype = ctypes.c_int64
    lib.raysh_mlp_get_params.argtypes = [P, P]
    lib.raysh_mlp_forward.argtypes = [P, P, ctypes.c_int32, P]
    lib.raysh_mlp_gradient.argtypes = [P, P, P, ctypes.c_int32, P, P]
    lib.raysh_mlp_adam_step.argtypes = [P, F, F, F, F]
    lib.raysh_mlp_train_step.argtypes = [P, P, P, ctypes.c_int32, F, F, F, F, P]
    lib.raysh_mlp_sync.argtypes = [P]
    lib.raysh_mlp_free.argtypes = [P]
    for name in ("raysh_mlp_create", "raysh_mlp_get_params", "raysh_mlp_forward", "raysh_mlp_gradient",
                 "raysh_mlp_adam_step", "raysh_mlp_train_step", "raysh_mlp_sync", "raysh_mlp_free"):
        getattr(lib, name).restype = I
    lib.raysh_autotune.argtypes = [P, ctypes.POINTER(Rays), ctypes.POINTER(Pixels), I, ctypes.c_char_p] + \
        [ctypes.POINTER(I)] * 4
    lib.raysh_autotune_batch.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(Rays), ctypes.POINTER(Pixels), I,
                                         ctypes.c_char_p] + [ctypes.POINTER(I)] * 4
    lib.raysh_autotune_batch.restype = I
    lib.raysh_shoot.argtypes = [P, ctypes.POINTER(Rays), I, P, P, ctypes.POINTER(Pixels), P]
    lib.raysh_map.argtypes = [P, ctypes.POINTER(Rays), ctypes.POINTER(Pixels), I, P,
                              ctypes.POINTER(ctypes.c_uint64)]
    lib.raysh_map_split_noalloc.argtypes = [P, ctypes.POINTER(Rays), ctypes.POINTER(Pixels), I, P]
    lib.raysh_map_split_noalloc.restype = I
    lib.raysh_map_batch.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(Rays),
                                    ctypes.POINTER(Pixels), I, ctypes.POINTER(P)]
    lib.raysh_sync.argtypes = [P]
    lib.raysh_free.argtypes = [P]
    lib.raysh_last_error.restype = ctypes.c_char_p
    for name in ("raysh_init", "raysh_set_stream", "raysh_set_tile", "raysh_get_tile", "raysh_autotune",
                 "raysh_shoot", "raysh_map", "raysh_map_batch", "raysh_sync", "raysh_free"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def check(code):
    if code != OK:
        raise RayshError(code, load().raysh_last_error().decode())


def rays_struct(r) -> Rays:
    """From a workloads.RayGrid, a tuple (x0, y0, dx, dy, nx, ny, i0, j0) or Rays."""
    if isinstance(r, Rays):
        return r
    t = r.as_tuple() if hasattr(r, "as_tuple") else tuple(r)
    return Rays(float(t[0]), float(t[1]), float(t[2]), float(t[3]),
                int(t[4]), int(t[5]), int(t[6]), int(t[7]))


def pixels_struct(p) -> Pixels:
    """From a workloads.PixelGrid, a tuple (X0, Y0, Px, Py, NX, NY) or Pixels."""
    if p is None or isinstance(p, Pixels):
        return p
    t = p.as_tuple() if hasattr(p, "as_tuple") else tuple(p)
    return Pixels(float(t[0]), float(t[1]), float(t[2]), float(t[3]), int(t[4]), int(t[5]))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("raysh needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _stream_handle(torch, device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _lens_struct(lens):
    """(raysh_lens, the arrays it points into, n_stars, (kappa_c, gamma1,
    gamma2)) for a lens given as a tuple (kappa_c, gamma1, gamma2, x, y, m)
    or an object with as_tuple()."""
    if hasattr(lens, "as_tuple"):
        lens = lens.as_tuple()
    kc, g1, g2, x, y, m = lens
    arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, m)]
    n = len(arrays[0])
    if not (len(arrays[1]) == n and len(arrays[2]) == n):
        raise ValueError("star arrays differ in length")
    cl = Lens(float(kc), float(g1), float(g2), n, *(a.ctypes.data if n else None for a in arrays))
    return cl, arrays, n, (float(kc), float(g1), float(g2))


class Context:
    """A lens (kappa_c, gamma, stars) resident on one GPU (raysh_init)."""

    def __init__(self, lens, device: int = 0, stream=None):
        torch = _torch()
        lib = load()
        cl, keep, n, macro = _lens_struct(lens)
        self.device = int(device)
        self._ptr = ctypes.c_void_p()
        check(lib.raysh_init(ctypes.byref(self._ptr), ctypes.byref(cl), self.device,
                             _stream_handle(torch, self.device, stream)))
        del keep
        self.n_stars = n
        self.lens = macro

    def set_lens(self, lens):
        """raysh_set_lens: another lens (kappa_c, gamma, stars) in this
        context, without creating a new one."""
        cl, keep, n, macro = _lens_struct(lens)
        check(load().raysh_set_lens(self.handle, ctypes.byref(cl)))
        del keep
        self.n_stars = n
        self.lens = macro

    @property
    def handle(self):
        if not self._ptr:
            raise RuntimeError("context is closed")
        return self._ptr

    def set_stream(self, stream):
        torch = _torch()
        check(load().raysh_set_stream(self.handle, _stream_handle(torch, self.device, stream)))

    def set_tile(self, precision, cx, cy, share=0, star_tile=0):
        check(load().raysh_set_tile(self.handle, PRECISIONS[precision], cx, cy, share, star_tile))

    def set_expansion(self, theta_open):
        """raysh_set_expansion: far-star criterion of the expansion mode."""
        check(load().raysh_set_expansion(self.handle, float(theta_open)))

    def set_expansion_block(self, block):
        """raysh_set_expansion_block: tiles per side of the expansion mode's
        workgroups (0 = automatic, 1, 2 or 4)."""
        check(load().raysh_set_expansion_block(self.handle, int(block)))

    def set_expansion_cells(self, mode):
        """raysh_set_expansion_cells: star cells of the expansion mode's block
        pass ("auto", "always" or "never")."""
        check(load().raysh_set_expansion_cells(self.handle, CELL_MODES[mode]))

    def set_star_split(self, parts):
        """raysh_set_star_split: 1 = one pass, 0 = automatic, n = n parts."""
        check(load().raysh_set_star_split(self.handle, int(parts)))

    def get_tile(self, precision):
        v = [ctypes.c_int() for _ in range(4)]
        check(load().raysh_get_tile(self.handle, PRECISIONS[precision], *[ctypes.byref(a) for a in v]))
        return tuple(a.value for a in v)

    def autotune(self, rays, pix, precision="fp64", cache_path=None):
        """Time the compiled launch shapes on a sample of this block, keep
        the fastest (raysh_autotune); returns (cx, cy, share, star_tile)."""
        v = [ctypes.c_int() for _ in range(4)]
        cp = cache_path.encode() if cache_path else None
        check(load().raysh_autotune(self.handle, ctypes.byref(rays_struct(rays)),
                                    ctypes.byref(pixels_struct(pix)), PRECISIONS[precision], cp,
                                    *[ctypes.byref(a) for a in v]))
        return tuple(a.value for a in v)

    def shoot(self, rays, precision="fp64", pix=None, beta=True, bins=True):
        """Per-ray (beta_x, beta_y, bin) device tensors of shape (ny, nx);
        entries not requested are None."""
        torch = _torch()
        r = rays_struct(rays)
        p = pixels_struct(pix)
        shape = (int(r.ny), int(r.nx))
        dev = torch.device("cuda", self.device)
        bx = torch.empty(shape, dtype=torch.float64, device=dev) if beta else None
        by = torch.empty(shape, dtype=torch.float64, device=dev) if beta else None
        b = torch.empty(shape, dtype=torch.int32, device=dev) if (bins and p is not None) else None
        check(load().raysh_shoot(self.handle, ctypes.byref(r), PRECISIONS[precision],
                                 _ptr(bx), _ptr(by), ctypes.byref(p) if p is not None else None,
                                 _ptr(b)))
        return bx, by, b

    def map(self, rays, pix, precision="fp64", counts=None, n_binned=False):
        """Accumulate Algorithm 1's counts into `counts` (a new zero map when
        None); returns counts, or (counts, rays binned by this call)."""
        torch = _torch()
        r = rays_struct(rays)
        p = pixels_struct(pix)
        if counts is None:
            counts = torch.zeros((p.ny, p.nx), dtype=torch.int32, device=torch.device("cuda", self.device))
        if counts.dtype != torch.int32 or not counts.is_contiguous() or counts.numel() != p.nx * p.ny:
            raise ValueError("counts must be a contiguous int32 tensor of ny*nx elements")
        nb = ctypes.c_uint64(0)
        check(load().raysh_map(self.handle, ctypes.byref(r), ctypes.byref(p), PRECISIONS[precision],
                               _ptr(counts), ctypes.byref(nb) if n_binned else None))
        return (counts, int(nb.value)) if n_binned else counts

    def map_split_noalloc(self, rays, pix, parts, counts):
        """raysh_map_split_noalloc: FP64 counts added into the caller's
        `counts`, the star sum split in `parts` (0 = automatic), with the
        partial sums in the library's static device array (no allocation)."""
        r = rays_struct(rays)
        p = pixels_struct(pix)
        if counts.dtype.itemsize != 4 or not counts.is_contiguous() or counts.numel() != p.nx * p.ny:
            raise ValueError("counts must be a contiguous int32 tensor of ny*nx elements")
        check(load().raysh_map_split_noalloc(self.handle, ctypes.byref(r), ctypes.byref(p), int(parts),
                                             _ptr(counts)))
        return counts

    def sync(self):
        check(load().raysh_sync(self.handle))

    def close(self):
        if self._ptr:
            check(load().raysh_free(self._ptr))
            self._ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._ptr:
                load().raysh_free(self._ptr)
        except Exception:
            pass


def list_tiles(precision):
    """Launch shapes compiled into the library: tuples (cx, cy, share, star_tile)."""
    lib = load()
    n = lib.raysh_list_tiles(PRECISIONS[precision], None, 0)
    if n < 0:
        check(-n)
    buf = (ctypes.c_int32 * (4 * n))()
    lib.raysh_list_tiles(PRECISIONS[precision], buf, n)
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(n)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def map_batch(contexts, rays, pix, precision="fp64", counts=None):
    """raysh_map_batch over several contexts in one persistent launch.
    rays and pix are per-set sequences; counts a per-set list of int32
    device maps (new zero maps when None).  Returns the list of maps."""
    torch = _torch()
    n = len(contexts)
    R = (Rays * n)(*[rays_struct(r) for r in rays])
    P = (Pixels * n)(*[pixels_struct(p) for p in pix])
    if counts is None:
        counts = [torch.zeros((P[s].ny, P[s].nx), dtype=torch.int32,
                              device=torch.device("cuda", contexts[s].device)) for s in range(n)]
    H = (ctypes.c_void_p * n)(*[c.handle for c in contexts])
    C = (ctypes.c_void_p * n)(*[c.data_ptr() for c in counts])
    check(load().raysh_map_batch(H, n, R, P, PRECISIONS[precision], C))
    return counts


def autotune_batch(contexts, rays, pix, precision="fp64", cache_path=None):
    """raysh_autotune_batch: time the compiled launch shapes with the batch
    kernel on a sample of these sets, set the fastest in every context and
    return it as (cx, cy, share, star_tile)."""
    n = len(contexts)
    R = (Rays * n)(*[rays_struct(r) for r in rays])
    P = (Pixels * n)(*[pixels_struct(p) for p in pix])
    H = (ctypes.c_void_p * n)(*[c.handle for c in contexts])
    v = [ctypes.c_int() for _ in range(4)]
    cp = cache_path.encode() if cache_path else None
    check(load().raysh_autotune_batch(H, n, R, P, PRECISIONS[precision], cp, *[ctypes.byref(a) for a in v]))
    return tuple(a.value for a in v)


def source_map_shape(nx, ny, profile, size, px, py):
    """raysh_source_map_shape: half-widths (rx, ry) of a source profile."""
    rx, ry = ctypes.c_int32(), ctypes.c_int32()
    check(load().raysh_source_map_shape(int(nx), int(ny), PROFILES[profile], float(size), float(px), float(py),
                                        ctypes.byref(rx), ctypes.byref(ry)))
    return rx.value, ry.value


def source_map(counts, pix, norm, profile="gaussian", size=0.05, stream=None):
    """raysh_source_map: the map seen by a source of the given profile.
    counts: int32 device map (NY, NX) of the window pix.  Returns the FP64
    source map (NY - 2 ry, NX - 2 rx) and its own pixel grid
    (x0 + rx Px, y0 + ry Py, Px, Py, NX - 2 rx, NY - 2 ry)."""
    torch = _torch()
    p = pixels_struct(pix)
    assert counts.dtype == torch.int32 and counts.is_contiguous() and tuple(counts.shape) == (p.ny, p.nx)
    rx, ry = source_map_shape(p.nx, p.ny, profile, size, p.px, p.py)
    lib = load()
    dev = counts.device
    ws = torch.empty(lib.raysh_source_map_workspace(p.nx, p.ny), dtype=torch.uint8, device=dev)
    out = torch.empty((p.ny - 2 * ry, p.nx - 2 * rx), dtype=torch.float64, device=dev)
    check(lib.raysh_source_map(_ptr(counts), p.nx, p.ny, float(norm), PROFILES[profile], float(size), p.px, p.py,
                               _ptr(ws), ws.numel(), _ptr(out), _stream_handle(torch, dev, stream)))
    grid = (p.x0 + rx * p.px, p.y0 + ry * p.py, p.px, p.py, p.nx - 2 * rx, p.ny - 2 * ry)
    return out, grid


def track_order(grid, xa, ya, xb, yb, sorted_end_points=False, stream=None):
    """raysh_track_order: a visiting order (int32 device permutation) of the
    tracks in which neighbouring tracks read neighbouring parts of the map.
    With sorted_end_points, also the end points in that order (FP64
    [4, n_tracks]); returns (order, sorted) then."""
    torch = _torch()
    g = pixels_struct(grid)
    n = int(xa.numel())
    for a in (xa, ya, xb, yb):
        assert a.dtype == torch.float64 and a.is_contiguous() and int(a.numel()) == n
    lib = load()
    ws = torch.empty(max(1, lib.raysh_track_order_workspace(ctypes.byref(g))), dtype=torch.uint8, device=xa.device)
    order = torch.empty(n, dtype=torch.int32, device=xa.device)
    srt = torch.empty((4, n), dtype=torch.float64, device=xa.device) if sorted_end_points else None
    check(lib.raysh_track_order(ctypes.byref(g), n, _ptr(xa), _ptr(ya), _ptr(xb), _ptr(yb), _ptr(ws), ws.numel(),
                                _ptr(order), _ptr(srt), _stream_handle(torch, xa.device, stream)))
    return (order, srt) if sorted_end_points else order


def fma_probe(precision, n_blocks, n_iter, out=None, stream=None):
    """raysh_fma_probe: a kernel of exactly 8 * n_iter FMA instructions per
    wave (a measurement aid).  Returns the device array of n_blocks * 256
    values (FP64 for "fp64", FP32 for "fp32_bulk")."""
    torch = _torch()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    dtype = torch.float64 if prec == FP64 else torch.float32
    if out is None:
        out = torch.empty(int(n_blocks) * 256, dtype=dtype, device="cuda")
    assert out.dtype == dtype and out.is_contiguous() and out.numel() >= int(n_blocks) * 256
    check(load().raysh_fma_probe(prec, int(n_blocks), int(n_iter), _ptr(out),
                                 _stream_handle(torch, out.device, stream)))
    return out


def light_curves(mu_s, grid, xa, ya, xb, yb, n_samples, out=None, order=None, sorted=None, stream=None):
    """raysh_light_curves: tracks (xa, ya) -> (xb, yb) (FP64 device arrays)
    sampled at n_samples points across the source map mu_s of pixel grid
    `grid`, visited in `order` when given, with the end points read from
    `sorted` when given (see track_order).  Returns FP64 (n_tracks,
    n_samples), NaN outside the map; row t is track t."""
    torch = _torch()
    g = pixels_struct(grid)
    n = int(xa.numel())
    for a in (mu_s, xa, ya, xb, yb):
        assert a.dtype == torch.float64 and a.is_contiguous()
    assert tuple(mu_s.shape) == (g.ny, g.nx) and all(int(a.numel()) == n for a in (ya, xb, yb))
    if order is not None:
        assert order.dtype == torch.int32 and order.is_contiguous() and int(order.numel()) == n
    if sorted is not None:
        assert sorted.dtype == torch.float64 and sorted.is_contiguous() and tuple(sorted.shape) == (4, n)
    if out is None:
        out = torch.empty((n, int(n_samples)), dtype=torch.float64, device=mu_s.device)
    assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == n * int(n_samples)
    check(load().raysh_light_curves(_ptr(mu_s), ctypes.byref(g), n, int(n_samples), _ptr(xa), _ptr(ya),
                                    _ptr(xb), _ptr(yb), _ptr(order), _ptr(sorted), _ptr(out),
                                    _stream_handle(torch, mu_s.device, stream)))
    return out
