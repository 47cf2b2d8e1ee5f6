"""GPU parity of source maps and light curves against the FP64 oracle."""
import numpy as np
import pytest

from oracle import light_curves as OL
from paper_1703_09707_amd import raysh as R
from paper_1703_09707_amd import workloads as W

pytestmark = pytest.mark.gpu

SOURCE_RTOL = 1e-13   # Gaussian taps: exp() of the GPU and of numpy may differ by an ulp


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return t


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def small_map(torch):
    """The 256^2 map of the 100-star workload, on the GPU and on the host."""
    w = W.plain_fp64_small()
    with R.Context(w.lens) as ctx:
        counts = ctx.map(w.rays, w.pix, "fp64")
    norm = (w.rays.dx * w.rays.dy) / (w.pix.Px * w.pix.Py)
    return w, counts, counts.cpu().numpy(), norm


@pytest.mark.parametrize("profile,size_px", [("gaussian", 0.7), ("gaussian", 2.0), ("gaussian", 9.3),
                                             ("disk", 0.5), ("disk", 3.0), ("disk", 11.7)])
def test_source_map_matches_oracle(torch, small_map, profile, size_px):
    w, counts, host, norm = small_map
    size = size_px * w.pix.Px
    mu, grid = R.source_map(counts, w.pix, norm, profile, size)
    want = OL.source_map(host, norm, R.PROFILES[profile], size, w.pix.Px, w.pix.Py)
    assert grid == OL.source_grid(w.pix.as_tuple(), R.PROFILES[profile], size)
    got = mu.cpu().numpy()
    assert got.shape == want.shape
    if profile == "disk":
        np.testing.assert_array_equal(got, want)     # integer sums: bit-exact
    else:
        np.testing.assert_allclose(got, want, rtol=SOURCE_RTOL, atol=0)


def _edge_tracks(grid):
    """Tracks that leave the map, touch its far edges exactly, sit still, or
    run along an edge."""
    x0, y0, px, py, nx, ny = grid
    xl, xh = x0 + 0.5 * px, x0 + (nx - 0.5) * px
    yl, yh = y0 + 0.5 * py, y0 + (ny - 0.5) * py
    xm, ym = 0.5 * (xl + xh), 0.5 * (yl + yh)
    t = [(xl, yl, xh, yh), (xh, yh, xl, yl), (xl - px, ym, xh + px, ym), (xm, yl - 3 * py, xm, yh + 3 * py),
         (xm, ym, xm, ym), (xl, yh, xh, yh), (xh, yl, xh, yh), (xh + 1.0, ym, xh + 2.0, ym),
         (np.nan, ym, xm, ym)]
    return tuple(np.array(v, np.float64) for v in zip(*t))


@pytest.mark.parametrize("n_samples", [1, 2, 7, 63, 64, 256, 1000])
def test_light_curves_match_oracle_bit_exact(torch, small_map, n_samples):
    """Given the same source map, the curves are bit-identical to the
    oracle's, NaN pattern included (random and edge tracks, a sample count
    that is not a multiple of the block)."""
    w, counts, _, norm = small_map
    mu, grid = R.source_map(counts, w.pix, norm, "gaussian", 2.0 * w.pix.Px)
    rnd = W.light_curve_tracks(grid, 50, 1.5, seed=31)
    edge = _edge_tracks(grid)
    xa, ya, xb, yb = (np.concatenate([a, b]) for a, b in zip(rnd, edge))
    dev = [torch.from_numpy(a).cuda() for a in (xa, ya, xb, yb)]
    got = R.light_curves(mu, grid, *dev, n_samples).cpu().numpy()
    want = OL.light_curves(mu.cpu().numpy(), grid, xa, ya, xb, yb, n_samples)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(want))
    np.testing.assert_array_equal(got, want)
    assert np.isfinite(got[:50]).all()   # the random tracks stay inside


def test_light_curves_large_workload(torch):
    """2^20 tracks x 256 samples on the 1024^2 map of the large
    configuration (the launch the benchmark times): sampled tracks are
    bit-identical to the oracle's, and every curve is finite."""
    lw = W.light_curves_large()
    w = lw.maps
    norm = (w.rays.dx * w.rays.dy) / (w.pix.Px * w.pix.Py)
    with R.Context(w.lens) as ctx:
        _say("map fp64 (large)")
        counts = ctx.map(w.rays, w.pix, "fp64")
    mu, grid = R.source_map(counts, w.pix, norm, lw.profile, lw.size)
    tracks = W.light_curve_tracks(grid, lw.n_tracks, lw.length)
    dev = [torch.from_numpy(a).cuda() for a in tracks]
    _say("light curves (large)")
    order, srt = R.track_order(grid, *dev, sorted_end_points=True)
    curves = R.light_curves(mu, grid, *dev, lw.n_samples, order=order, sorted=srt)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(curves).all())
    rng = np.random.default_rng(5)
    sel = rng.integers(0, lw.n_tracks, 200)
    want = OL.light_curves(mu.cpu().numpy(), grid, *(a[sel] for a in tracks), lw.n_samples)
    got = curves[torch.as_tensor(sel, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(got, want)
    # the mean over many tracks approaches the map's mean magnification
    _say("mean of curves", float(curves.mean()), "mean of source map", float(mu.mean()))
    assert abs(float(curves.mean()) / float(mu.mean()) - 1) < 0.05


def test_light_curves_maximum_sizes(torch, small_map):
    """The largest sample count a track may have (2^24) in the track kernel,
    and 2^20 tracks of 63 samples in the one-lane-per-sample kernel, with and
    without the track order: sampled outputs are bit-identical to the
    oracle's."""
    w, counts, _, norm = small_map
    mu, grid = R.source_map(counts, w.pix, norm, "gaussian", 2.0 * w.pix.Px)
    host_mu = mu.cpu().numpy()
    x0, y0, px, py, nx, ny = grid
    xl, xh = x0 + 0.5 * px, x0 + (nx - 0.5) * px
    yl, yh = y0 + 0.5 * py, y0 + (ny - 0.5) * py
    ym = 0.5 * (yl + yh)
    # two tracks of 2^24 samples: corner to corner, and one that leaves the map
    xa, ya = np.array([xl, xl - 2 * px]), np.array([yl, ym])
    xb, yb = np.array([xh, xh + 2 * px]), np.array([yh, ym + 3 * py])
    n = 1 << 24
    _say("light curves: 2 tracks x 2^24 samples")
    got = R.light_curves(mu, grid, *(torch.from_numpy(a).cuda() for a in (xa, ya, xb, yb)), n)
    rng = np.random.default_rng(11)
    ks = np.unique(np.concatenate([[0, 1, 255, 256, 257, n - 257, n - 256, n - 2, n - 1],
                                   rng.integers(0, n, 3000)]))
    u, v = OL.sample_indices(grid, xa, ya, xb, yb, n)
    want = OL.interpolate_indices(host_mu, u[:, ks], v[:, ks])
    g = got[:, torch.as_tensor(ks, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(np.isnan(g), np.isnan(want))
    np.testing.assert_array_equal(g, want)
    assert np.isfinite(g[0]).all() and np.isnan(g[1]).any() and np.isfinite(g[1]).any()
    del got
    # 2^20 short tracks: the kernel that takes one lane per sample
    n_tracks, n_short = 1 << 20, 63
    tracks = W.light_curve_tracks(grid, n_tracks, 1.5, seed=77)
    dev = [torch.from_numpy(a).cuda() for a in tracks]
    _say("light curves: 2^20 tracks x 63 samples")
    plain = R.light_curves(mu, grid, *dev, n_short)
    order, srt = R.track_order(grid, *dev, sorted_end_points=True)
    ordered = R.light_curves(mu, grid, *dev, n_short, order=order, sorted=srt)
    assert bool(torch.isfinite(plain).all())
    assert torch.equal(plain, ordered)
    sel = rng.integers(0, n_tracks, 300)
    want = OL.light_curves(host_mu, grid, *(a[sel] for a in tracks), n_short)
    np.testing.assert_array_equal(plain[torch.as_tensor(sel, device="cuda")].cpu().numpy(), want)


def test_source_map_and_light_curve_errors(torch, small_map):
    w, counts, _, norm = small_map
    with pytest.raises(R.RayshError):
        R.source_map(counts, w.pix, norm, "disk", 200 * w.pix.Px)        # larger than the map
    mu, grid = R.source_map(counts, w.pix, norm, "disk", 2 * w.pix.Px)
    host = np.zeros(4)
    lib = R.load()
    g = R.pixels_struct(grid)
    import ctypes
    code = lib.raysh_light_curves(ctypes.c_void_p(mu.data_ptr()), ctypes.byref(g), 4, 8,
                                  host.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(mu.data_ptr()),
                                  ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(mu.data_ptr()), None, None,
                                  ctypes.c_void_p(mu.data_ptr()), None)
    assert code == R.EINVAL and "xa" in lib.raysh_last_error().decode()
    tiny = torch.zeros(3, dtype=torch.float64, device="cuda")
    t = ctypes.c_void_p(tiny.data_ptr())
    code = lib.raysh_light_curves(ctypes.c_void_p(mu.data_ptr()), ctypes.byref(g), 1 << 26, 8, t, t, t, t, None,
                                  None, ctypes.c_void_p(mu.data_ptr()), None)     # 512 MiB per track array
    assert code == R.EINVAL and "needed" in lib.raysh_last_error().decode()
    assert int(tiny.abs().sum()) == 0
    n4 = torch.zeros(4, dtype=torch.float64, device="cuda")
    p4 = ctypes.c_void_p(n4.data_ptr())
    code = lib.raysh_light_curves(ctypes.c_void_p(mu.data_ptr()), ctypes.byref(g), 4, 8, p4, p4, p4, p4,
                                  host.ctypes.data_as(ctypes.c_void_p), None, ctypes.c_void_p(mu.data_ptr()), None)
    assert code == R.EINVAL and "order" in lib.raysh_last_error().decode()
    s16 = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    code = lib.raysh_light_curves(ctypes.c_void_p(mu.data_ptr()), ctypes.byref(g), 4, 8, p4, p4, p4, p4, None,
                                  ctypes.c_void_p(s16.data_ptr()), ctypes.c_void_p(mu.data_ptr()), None)
    assert code == R.EINVAL and "sorted" in lib.raysh_last_error().decode()


def test_track_order(torch, small_map):
    """The order is a permutation that visits tracks region by region
    (consecutive tracks' midpoints are far closer than in the given order),
    and the curves do not depend on it, for both kernels (fewer than 64
    samples: one lane per sample; more: one wave per track chunk)."""
    w, counts, _, norm = small_map
    mu, grid = R.source_map(counts, w.pix, norm, "gaussian", 2.0 * w.pix.Px)
    tracks = W.light_curve_tracks(grid, 20000, 1.0, seed=41)
    dev = [torch.from_numpy(a).cuda() for a in tracks]
    order = R.track_order(grid, *dev)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(len(o)))
    mx, my = 0.5 * (tracks[0] + tracks[2]), 0.5 * (tracks[1] + tracks[3])
    step = lambda idx: np.hypot(np.diff(mx[idx]), np.diff(my[idx])).mean()   # noqa: E731
    _say("mean step between consecutive midpoints: given", step(np.arange(len(o))), "ordered", step(o))
    assert step(o) < 0.1 * step(np.arange(len(o)))
    order2, srt = R.track_order(grid, *dev, sorted_end_points=True)
    o2 = order2.cpu().numpy()
    assert np.array_equal(np.sort(o2), np.arange(len(o2)))
    assert np.array_equal(srt.cpu().numpy(), np.stack([a[o2] for a in tracks]))
    for n_samples in (7, 300):
        plain = R.light_curves(mu, grid, *dev, n_samples)
        for kw in (dict(order=order), dict(order=order2, sorted=srt)):
            ordered = R.light_curves(mu, grid, *dev, n_samples, **kw)
            assert torch.equal(torch.isnan(plain), torch.isnan(ordered))
            assert torch.equal(torch.nan_to_num(plain, nan=-1.0), torch.nan_to_num(ordered, nan=-1.0))


def _cell_keys(grid, tracks):
    """Each track's sort key as the header states it: the Morton number of
    the 16 x 16-pixel cell (cells doubled while more than 2048 a side)
    holding the midpoint of its end points, midpoints outside the map
    clamped to the nearest edge cell."""
    x0, y0, px, py, nx, ny = grid
    cell = 16
    while (max(nx, ny) + cell - 1) // cell > 2048:
        cell *= 2
    cx_n, cy_n = (nx + cell - 1) // cell, (ny + cell - 1) // cell
    mx, my = 0.5 * (tracks[0] + tracks[2]), 0.5 * (tracks[1] + tracks[3])

    def cells(m, o, ip, n):
        c = ((m - o) * ip) / float(cell)
        with np.errstate(invalid="ignore"):
            k = np.where(c >= 0.0, np.minimum(c, n - 1), 0.0)
        return np.where(np.isnan(c), 0, np.floor(k)).astype(np.int64)

    cx, cy = cells(mx, x0, 1.0 / px, cx_n), cells(my, y0, 1.0 / py, cy_n)
    key = np.zeros(len(mx), np.int64)
    for b in range(12):
        key |= ((cx >> b) & 1) << (2 * b) | ((cy >> b) & 1) << (2 * b + 1)
    return key


@pytest.mark.parametrize("side", [1012, 4096])
def test_track_order_sorted_by_cell(torch, side):
    """The order visits cells in Morton order, every track in its
    midpoint's cell, for a map of 64 x 64 cells (counters a cache line
    apart) and one of 256 x 256 (counters packed); tracks beyond the map
    edges go to the edge cells."""
    grid = (-5.0, -4.0, 10.0 / side, 8.0 / side, side, side)
    rng = np.random.default_rng(side)
    n = 300_000
    mid_x, mid_y = rng.uniform(-5.5, 5.5, n), rng.uniform(-4.5, 4.5, n)   # some midpoints off the map
    ang, half = rng.uniform(0, 2 * np.pi, n), rng.uniform(0.0, 0.5, n)
    tracks = [mid_x - half * np.cos(ang), mid_y - half * np.sin(ang),
              mid_x + half * np.cos(ang), mid_y + half * np.sin(ang)]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in tracks]
    order, srt = R.track_order(grid, *dev, sorted_end_points=True)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(n))
    keys = _cell_keys(grid, tracks)[o]
    assert np.all(np.diff(keys) >= 0)
    assert np.array_equal(srt.cpu().numpy(), np.stack([a[o] for a in tracks]))


def test_track_order_entries_outside_are_skipped(torch, small_map):
    w, counts, _, norm = small_map
    mu, grid = R.source_map(counts, w.pix, norm, "disk", 2.0 * w.pix.Px)
    tracks = W.light_curve_tracks(grid, 6, 1.0, seed=42)
    dev = [torch.from_numpy(a).cuda() for a in tracks]
    order = torch.tensor([5, -1, 0, 6, 1 << 30, 2], dtype=torch.int32, device="cuda")
    for n_samples in (5, 100):
        out = torch.full((6, n_samples), 1234.5, dtype=torch.float64, device="cuda")
        R.light_curves(mu, grid, *dev, n_samples, out=out, order=order)
        full = R.light_curves(mu, grid, *dev, n_samples)
        for t in (0, 2, 5):
            assert torch.equal(out[t], full[t])
        for t in (1, 3, 4):
            assert bool((out[t] == 1234.5).all())


@pytest.mark.parametrize("nx,ny", [(256, 256), (300, 3), (3, 300), (7, 5), (1024, 40)])
def test_light_curves_all_directions_and_steps(torch, nx, ny):
    """Tracks in 16 directions with steps from a tenth of a pixel to nearly a
    pixel, crossing the map's edges and corners, on square, thin and tiny
    maps, in chunks that end inside a wave: bit-identical to the oracle's."""
    rng = np.random.default_rng(nx * 1000 + ny)
    mu_h = rng.uniform(0.1, 10.0, (ny, nx))
    mu = torch.from_numpy(mu_h).cuda()
    px, py = 0.013, 0.017
    grid = (-0.4, 0.25, px, py, nx, ny)
    xs, ys, xe, ye = [], [], [], []
    for n in (64, 256, 257, 1000):
        for d in range(16):
            phi = 2 * np.pi * d / 16 + 0.01
            for step in (0.1, 0.45, 0.499, 0.5, 0.501, 0.9):
                length = step * (n - 1)   # in pixels along the major axis
                c, s = np.cos(phi), np.sin(phi)
                scale = length / max(abs(c), abs(s))
                x0 = grid[0] + rng.uniform(-0.2, 1.2) * nx * px
                y0 = grid[1] + rng.uniform(-0.2, 1.2) * ny * py
                xs.append(x0)
                ys.append(y0)
                xe.append(x0 + scale * c * px)
                ye.append(y0 + scale * s * py)
        xa, ya, xb, yb = (np.array(v, np.float64) for v in (xs, ys, xe, ye))
        dev = [torch.from_numpy(a).cuda() for a in (xa, ya, xb, yb)]
        got = R.light_curves(mu, grid, *dev, n).cpu().numpy()
        want = OL.light_curves(mu_h, grid, xa, ya, xb, yb, n)
        np.testing.assert_array_equal(np.isnan(got), np.isnan(want))
        np.testing.assert_array_equal(got, want)
        xs, ys, xe, ye = [], [], [], []
