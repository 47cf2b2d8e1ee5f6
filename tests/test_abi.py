"""The C-ABI library: loads, exports what include/raysh.h declares, and
rejects bad arguments before touching a device (CPU only)."""
import ctypes
import math
import os
import re

import pytest

from paper_1703_09707_amd import raysh as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "raysh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(raysh_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return R.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(R.EXPORTS)


def test_compiled_tile_lists():
    f64 = R.list_tiles("fp64")
    f32 = R.list_tiles("fp32_bulk")
    assert len(f64) >= 5 and len(f32) >= 5
    # FP64: share in (2, 4, 8, 16) r^2 values per reciprocal, of which t[3]
    # (1, 2 or 4) are consecutive stars; the rest are rays of the lane
    assert all(t[2] in (2, 4, 8, 16) and t[3] in (1, 2, 4) and t[2] % t[3] == 0 for t in f64)
    assert all(t[2] // t[3] <= t[0] * t[1] for t in f64)
    assert all(t[2] == 0 and t[3] > 0 for t in f32)
    lib = R.load()
    assert lib.raysh_list_tiles(5, None, 0) == -R.EINVAL


def test_struct_layouts():
    assert ctypes.sizeof(R.Lens) == 56
    assert ctypes.sizeof(R.Rays) == 64
    assert ctypes.sizeof(R.Pixels) == 40


def _err(lib):
    return lib.raysh_last_error().decode()


def _init(lib, kc=0.1, g1=0.2, g2=0.0, xs=(0.0,), ys=(0.0,), ms=(1.0,), n=None):
    arr = ctypes.c_double * max(len(xs), 1)
    x, y, m = arr(*xs), arr(*ys), arr(*ms)
    lens = R.Lens(kc, g1, g2, len(xs) if n is None else n, ctypes.addressof(x), ctypes.addressof(y),
                  ctypes.addressof(m))
    out = ctypes.c_void_p()
    code = lib.raysh_init(ctypes.byref(out), ctypes.byref(lens), 0, None)
    return code, out


@pytest.mark.parametrize("kw,code,msg", [
    (dict(kc=math.nan), R.EINVAL, "finite"),
    (dict(g2=math.inf), R.EINVAL, "finite"),
    (dict(n=-1), R.EINVAL, "n_stars"),
    (dict(n=2 ** 31), R.EOVERFLOW, "n_stars"),
    (dict(xs=(math.nan,)), R.EINVAL, "position"),
    (dict(ys=(math.inf,)), R.EINVAL, "position"),
    (dict(ms=(-1.0,)), R.EINVAL, "mass"),
    (dict(ms=(math.nan,)), R.EINVAL, "mass"),
])
def test_init_rejects_bad_lens(lib, kw, code, msg):
    got, out = _init(lib, **kw)
    assert got == code
    assert msg in _err(lib)
    assert not out.value


def test_init_null_arguments(lib):
    lens = R.Lens(0.0, 0.0, 0.0, 0, None, None, None)
    assert lib.raysh_init(None, ctypes.byref(lens), 0, None) == R.EINVAL
    out = ctypes.c_void_p()
    assert lib.raysh_init(ctypes.byref(out), None, 0, None) == R.EINVAL
    lens = R.Lens(0.0, 0.0, 0.0, 3, None, None, None)
    assert lib.raysh_init(ctypes.byref(out), ctypes.byref(lens), 0, None) == R.EINVAL
    assert "NULL" in _err(lib)
    lens = R.Lens(0.0, 0.0, 0.0, 0, None, None, None)
    assert lib.raysh_init(ctypes.byref(out), ctypes.byref(lens), -1, None) == R.EINVAL


GOOD_RAYS = R.Rays(-1.0, -1.0, 0.01, 0.01, 200, 200, 0, 0)
GOOD_PIX = R.Pixels(-1.0, -1.0, 0.1, 0.1, 20, 20)


@pytest.mark.parametrize("rays,code,msg", [
    (R.Rays(math.nan, 0, 0.1, 0.1, 4, 4, 0, 0), R.EINVAL, "origin"),
    (R.Rays(0, 0, 0.0, 0.1, 4, 4, 0, 0), R.EINVAL, "spacing"),
    (R.Rays(0, 0, 0.1, -0.1, 4, 4, 0, 0), R.EINVAL, "spacing"),
    (R.Rays(0, 0, math.inf, 0.1, 4, 4, 0, 0), R.EINVAL, "spacing"),
    (R.Rays(0, 0, 0.1, 0.1, -4, 4, 0, 0), R.EINVAL, "counts"),
    (R.Rays(0, 0, 0.1, 0.1, 4, 4, -1, 0), R.EINVAL, "offsets"),
    (R.Rays(0, 0, 0.1, 0.1, 65536, 32768, 0, 0), R.EOVERFLOW, "2^31"),
    (R.Rays(0, 0, 0.1, 0.1, 4, 4, 2 ** 53, 0), R.EOVERFLOW, "2^53"),
    (R.Rays(0, 0, 1e305, 0.1, 4, 4, 2 ** 20, 0), R.EINVAL, "not finite"),
])
def test_shoot_and_map_reject_bad_rays(lib, rays, code, msg):
    assert lib.raysh_shoot(None, ctypes.byref(rays), 0, None, None, ctypes.byref(GOOD_PIX), None) == code
    assert msg in _err(lib)
    dummy = ctypes.c_void_p(1)
    assert lib.raysh_map(None, ctypes.byref(rays), ctypes.byref(GOOD_PIX), 0, dummy, None) == code


@pytest.mark.parametrize("pix,code,msg", [
    (R.Pixels(math.nan, 0, 0.1, 0.1, 4, 4), R.EINVAL, "origin"),
    (R.Pixels(0, 0, 0.0, 0.1, 4, 4), R.EINVAL, "pixel size"),
    (R.Pixels(0, 0, 0.1, 0.1, 0, 4), R.EINVAL, "pixel counts"),
    (R.Pixels(0, 0, 0.1, 0.1, 4, -4), R.EINVAL, "pixel counts"),
    (R.Pixels(0, 0, 0.1, 0.1, 65536, 65536), R.EOVERFLOW, "pixels"),
    (R.Pixels(1e308, 0, 1e308, 0.1, 4, 4), R.EINVAL, "not finite"),
])
def test_map_rejects_bad_window(lib, pix, code, msg):
    dummy = ctypes.c_void_p(1)
    assert lib.raysh_map(None, ctypes.byref(GOOD_RAYS), ctypes.byref(pix), 0, dummy, None) == code
    assert msg in _err(lib)


def test_other_argument_errors(lib):
    dummy = ctypes.c_void_p(1)
    r, p = ctypes.byref(GOOD_RAYS), ctypes.byref(GOOD_PIX)
    assert lib.raysh_map(None, r, p, 7, dummy, None) == R.EINVAL
    assert "precision" in _err(lib)
    assert lib.raysh_map(None, r, p, 0, None, None) == R.EINVAL
    assert "counts" in _err(lib)
    assert lib.raysh_map(None, r, p, 0, dummy, None) == R.EINVAL
    assert "ctx" in _err(lib)
    assert lib.raysh_shoot(None, r, 0, None, None, None, dummy) == R.EINVAL
    assert "window" in _err(lib)
    assert lib.raysh_map(None, None, p, 0, dummy, None) == R.EINVAL
    assert lib.raysh_map(None, r, None, 0, dummy, None) == R.EINVAL
    assert lib.raysh_map_batch(None, 1, None, None, 0, None) == R.EINVAL
    sets = (ctypes.c_void_p * 1)(None)
    rays = (R.Rays * 1)(GOOD_RAYS)
    pix = (R.Pixels * 1)(GOOD_PIX)
    cnt = (ctypes.c_void_p * 1)(1)
    assert lib.raysh_map_batch(sets, 0, rays, pix, 0, cnt) == R.EINVAL
    assert lib.raysh_map_batch(sets, 1, rays, pix, 0, cnt) == R.EINVAL
    assert "context" in _err(lib)
    assert lib.raysh_set_tile(None, 0, 2, 4, 2, 0) == R.EINVAL
    assert lib.raysh_autotune(None, r, p, 0, None, None, None, None, None) == R.EINVAL
    assert "ctx" in _err(lib)
    assert lib.raysh_sync(None) == R.EINVAL
    assert lib.raysh_set_star_split(None, 2) == R.EINVAL
    assert lib.raysh_set_expansion(None, 0.25) == R.EINVAL
    assert lib.raysh_set_expansion_block(None, 1) == R.EINVAL
    assert lib.raysh_set_expansion_cells(None, 0) == R.EINVAL
    assert lib.raysh_expansion_order() >= 16
    assert lib.raysh_list_tiles(2, None, 0) == -R.EINVAL
    assert lib.raysh_free(None) == R.OK
    assert lib.raysh_n_stars(None) == 0


def test_python_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError, match="GPU"):
        R.Context((0.0, 0.0, 0.0, [], [], []))


def test_histogram_and_mlp_argument_errors(lib):
    D = 1.0
    dummy = ctypes.c_void_p(1)
    h = lib.raysh_log_mag_histogram
    assert lib.raysh_histogram_workspace(0, 5) == 0
    assert lib.raysh_histogram_workspace(10, 10) >= 800
    args = dict(nx=64, ny=64, norm=0.5, sigma=0.1, px=0.1, py=0.1, mu_ref=1.0, nbins=64, lo=-2.0, hi=2.0)

    def call(**kw):
        a = dict(args, **kw)
        return h(dummy, a["nx"], a["ny"], a["norm"], a["sigma"], a["px"], a["py"], a["mu_ref"],
                 a["nbins"], a["lo"], a["hi"], dummy, 1 << 20, dummy, None, None)
    for kw, msg in [(dict(nx=0), "map size"), (dict(norm=-1.0), "norm"), (dict(sigma=math.nan), "sigma"),
                    (dict(px=0.0), "pixel"), (dict(mu_ref=0.0), "mu_ref"), (dict(nbins=0), "nbins"),
                    (dict(lo=2.0, hi=-2.0), "range"), (dict(sigma=5.0), "larger than the map"),
                    (dict(nx=65536, ny=65536), "2^31")]:
        code = call(**kw)
        assert code in (R.EINVAL, R.EOVERFLOW) and msg in _err(lib), (kw, _err(lib))
    assert h(dummy, 64, 64, D, 0.1, 0.1, 0.1, D, 64, -2.0, 2.0, dummy, 16, dummy, None, None) == R.EINVAL
    assert "workspace" in _err(lib)
    out = ctypes.c_void_p()
    p = (ctypes.c_float * 10)()
    assert lib.raysh_mlp_create(ctypes.byref(out), 0, None, 0, 4, 4, 8, p) == R.EINVAL
    assert lib.raysh_mlp_create(ctypes.byref(out), 0, None, 4, 4, 4, 8, None) == R.EINVAL
    assert lib.raysh_mlp_create(None, 0, None, 4, 4, 4, 8, p) == R.EINVAL
    nan = (ctypes.c_float * 64)(*([0.0] * 10 + [math.nan] + [0.0] * 53))   # 52 parameters
    assert lib.raysh_mlp_create(ctypes.byref(out), 0, None, 2, 4, 4, 8, nan) == R.EINVAL
    assert "not finite" in _err(lib)
    assert lib.raysh_mlp_forward(None, dummy, 4, dummy) == R.EINVAL
    assert lib.raysh_mlp_adam_step(None, 1e-3, 0.9, 0.999, 1e-8) == R.EINVAL
    assert lib.raysh_mlp_free(None) == R.OK
    assert lib.raysh_mlp_n_params(None) == 0


@pytest.mark.parametrize("profile,size,px,py", [(0, 0.05, 0.03125, 0.0625), (0, 0.1, 0.0195, 0.0195),
                                                (1, 1.375, 0.5, 0.25), (1, 3.0, 1.0, 1.0),
                                                (1, 0.3, 0.125, 0.0625), (1, 0.01, 0.1, 0.1)])
def test_source_map_shape_matches_oracle(lib, profile, size, px, py):
    """The library's source half-widths (host code) equal the oracle's."""
    from oracle import light_curves as LC
    rx, ry = R.source_map_shape(200, 150, profile, size, px, py)
    assert (rx, ry) == LC.source_radii(profile, size, px, py)


def test_source_map_and_light_curve_argument_errors(lib):
    dummy = ctypes.c_void_p(1)
    rx, ry = ctypes.c_int32(), ctypes.c_int32()
    s = lib.raysh_source_map_shape
    for args, msg in [((64, 64, 2, 0.1, 0.1, 0.1), "profile"), ((0, 64, 0, 0.1, 0.1, 0.1), "map size"),
                      ((64, 64, 0, -0.1, 0.1, 0.1), "source size"), ((64, 64, 1, math.nan, 0.1, 0.1), "source size"),
                      ((64, 64, 0, 0.1, 0.0, 0.1), "pixel"), ((64, 64, 0, 3.0, 0.1, 0.1), "larger than the map"),
                      ((64, 64, 1, 6.5, 0.1, 0.1), "larger than the map"), ((64, 64, 1, 3.2, 0.1, 0.1), "2 x 2")]:
        assert s(*args, ctypes.byref(rx), ctypes.byref(ry)) == R.EINVAL, args
        assert msg in _err(lib), (args, _err(lib))
    assert s(64, 64, 1, 0.25, 0.1, 0.1, None, None) == R.OK
    assert lib.raysh_source_map_workspace(0, 4) == 0
    assert lib.raysh_source_map_workspace(10, 10) >= 8 * 100
    sm = lib.raysh_source_map
    assert sm(dummy, 64, 64, 0.0, 0, 0.1, 0.1, 0.1, dummy, 1 << 20, dummy, None) == R.EINVAL
    assert "norm" in _err(lib)
    assert sm(None, 64, 64, 1.0, 0, 0.1, 0.1, 0.1, dummy, 1 << 20, dummy, None) == R.EINVAL
    assert sm(dummy, 64, 64, 1.0, 0, 0.1, 0.1, 0.1, dummy, 16, dummy, None) == R.EINVAL
    assert "workspace" in _err(lib)
    lc = lib.raysh_light_curves
    g = R.Pixels(0.0, 0.0, 0.1, 0.1, 16, 16)
    d = dummy
    assert lc(d, None, 4, 8, d, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(d, ctypes.byref(R.Pixels(0.0, 0.0, 0.1, 0.1, 1, 16)), 4, 8, d, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(d, ctypes.byref(g), -1, 8, d, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(d, ctypes.byref(g), 4, 0, d, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(d, ctypes.byref(g), 4, (1 << 24) + 1, d, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(d, ctypes.byref(g), 1 << 40, 1 << 20, d, d, d, d, None, None, d, None) == R.EOVERFLOW
    assert lc(d, ctypes.byref(g), 4, 8, None, d, d, d, None, None, d, None) == R.EINVAL
    assert lc(None, ctypes.byref(g), 0, 8, None, None, None, None, None, None, None, None) == R.OK   # no tracks: no-op
    to = lib.raysh_track_order
    assert lib.raysh_track_order_workspace(None) == 0
    assert lib.raysh_track_order_workspace(ctypes.byref(R.Pixels(0.0, 0.0, 0.1, 0.1, 0, 16))) == 0
    # 1012 pixels a side: 64 cells of 16 pixels, Morton keys over 64 x 64,
    # their counters a 128-byte line (32 words) apart
    assert lib.raysh_track_order_workspace(ctypes.byref(R.Pixels(0.0, 0.0, 0.1, 0.1, 1012, 1012))) == \
        4 * (64 * 64 * 32 + 1)
    # 2896 pixels a side: 181 cells, keys over 256 x 256 (65536 > 32768): counters packed
    assert lib.raysh_track_order_workspace(ctypes.byref(R.Pixels(0.0, 0.0, 0.1, 0.1, 2896, 2896))) == \
        4 * (256 * 256 + 1)
    # 40000 pixels a side: cells grow to 32 pixels (1250 a side), keys over 2048 x 2048
    assert lib.raysh_track_order_workspace(ctypes.byref(R.Pixels(0.0, 0.0, 0.1, 0.1, 40000, 100))) == \
        4 * (2048 * 2048 + 1)
    assert to(None, 4, d, d, d, d, d, 1 << 30, d, None, None) == R.EINVAL
    assert to(ctypes.byref(g), -1, d, d, d, d, d, 1 << 30, d, None, None) == R.EINVAL
    assert to(ctypes.byref(g), 1 << 31, d, d, d, d, d, 1 << 30, d, None, None) == R.EOVERFLOW
    assert to(ctypes.byref(g), 4, d, d, d, d, d, 4, d, None, None) == R.EINVAL
    assert "workspace" in _err(lib)
    assert to(ctypes.byref(g), 4, d, None, d, d, d, 1 << 30, d, None, None) == R.EINVAL
    assert to(ctypes.byref(g), 0, None, None, None, None, None, 0, None, None, None) == R.OK


def test_fma_probe_argument_errors(lib):
    d = ctypes.c_void_p(1)
    assert lib.raysh_fma_probe(R.FP64_EXPANSION, 1, 1, d, None) == R.EINVAL
    assert "precision" in _err(lib)
    assert lib.raysh_fma_probe(R.FP64, 0, 1, d, None) == R.EINVAL
    assert lib.raysh_fma_probe(R.FP32_BULK, 1 << 31, 1, d, None) == R.EINVAL
    assert lib.raysh_fma_probe(R.FP64, 1, 0, d, None) == R.EINVAL
    assert "n_iter" in _err(lib)
    assert lib.raysh_fma_probe(R.FP64, 1, 1, None, None) == R.EINVAL


def test_set_lens_argument_errors(lib):
    assert lib.raysh_set_lens(None, None) == R.EINVAL
    assert "ctx" in _err(lib)
