"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar (FP64): |beta_gpu - beta_oracle| <= 1e-12 S per ray, S = |theta| +
|K theta| + sum_k m_k/r_k (the scale rounding errors of Eq. (1) follow), and
every ray in the oracle's pixel except those whose oracle beta lies within
1e-12 S of a pixel edge (there either pixel is within the beta bar; such
rays are counted and are rare).  FP32-bulk: at most 1e-4 of rays in a
different pixel than FP64.  Integer invariants (band additivity, map =
histogram of bins, batch = single) are exact.
"""
import json
import os

import numpy as np
import pytest

from oracle import shooter as ora
from paper_1703_09707_amd import raysh as R
from paper_1703_09707_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_SHAPES = [tuple(t) for t in R.list_tiles("fp64")]             # (cx, cy, share, stars per group)
FP32_SHAPES = [(t[0], t[1], t[3]) for t in R.list_tiles("fp32_bulk")]  # (cx, cy, star_tile)
BETA_TOL = 1e-12
MISBIN_FP64 = 1e-6
MISBIN_FP32 = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return t


def _np(t):
    return t.cpu().numpy()


def _say(*a):
    print(*a, flush=True)


def _set64(ctx, shape):
    ctx.set_tile("fp64", shape[0], shape[1], share=shape[2], star_tile=shape[3])


def _near_edges(bx, by, s, pix):
    """Rays whose (oracle) beta lies within BETA_TOL * S of a pixel edge of
    the window's grid (window edges included): within the beta bar of an
    edge, either pixel is a correct answer."""
    X0, Y0, Px, Py = (float(v) for v in pix[:4])
    with np.errstate(invalid="ignore"):
        u = (np.asarray(bx) - X0) / Px
        v = (np.asarray(by) - Y0) / Py
        du = np.abs(u - np.round(u)) * Px
        dv = np.abs(v - np.round(v)) * Py
        tol = BETA_TOL * np.asarray(s)
        near = (du <= tol) | (dv <= tol)
    return near & np.isfinite(bx) & np.isfinite(by)


def _assert_bins(got, want, near, what=""):
    """Every ray in the oracle's pixel, except rays in the edge band."""
    got, want, near = np.asarray(got).ravel(), np.asarray(want).ravel(), np.asarray(near).ravel()
    bad = np.count_nonzero((got != want) & ~near)
    assert bad == 0, f"{what}: {bad} rays binned differently from the oracle away from pixel edges"
    return int(np.count_nonzero(near))


def _assert_map(got, want_counts, want_n, got_n, n_near, what=""):
    """A map against the oracle's: they differ by at most the edge-band rays
    (each moves one count), and are equal when there are none."""
    d = 0.5 * (np.abs(np.asarray(got, np.int64) - want_counts).sum() + abs(got_n - want_n))
    assert d <= n_near, f"{what}: maps differ by {d} rays, {n_near} near pixel edges"


# ----------------------------------------------------------------- exact fixtures
def test_golden_exact_tiny(torch):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_tiny.json")))
    L, Rr, P = g["lens"], g["rays"], g["pix"]
    lens = (L["kappa_c"], L["gamma1"], L["gamma2"], L["x"], L["y"], L["m"])
    rays = tuple(Rr[k] for k in ("x0", "y0", "dx", "dy", "nx", "ny", "i0", "j0"))
    pix = tuple(P[k] for k in ("X0", "Y0", "Px", "Py", "NX", "NY"))
    want = np.array(g["bins"])
    near = np.array(g["edge_distance"]) < 1e-9
    with R.Context(lens) as ctx:
        for shape in FP64_SHAPES:
            _set64(ctx, shape)
            _, _, b = ctx.shoot(rays, "fp64", pix)
            got = _np(b).ravel()
            np.testing.assert_array_equal(got[~near], want[~near])
            assert got[want == -1].tolist() == want[want == -1].tolist()
            counts = _np(ctx.map(rays, pix, "fp64")).ravel()
            if not near.any():
                np.testing.assert_array_equal(counts, np.array(g["counts"]))


@pytest.mark.parametrize("kc,g1,g2", [(0.25, 0.125, 0.0625), (0.5, -0.25, 0.1875),
                                      (1.0, 0.0, 0.0), (0.75, 0.25, 0.0)])
def test_dyadic_sheet_exact(torch, kc, g1, g2):
    """No stars: every beta and pixel is exact, so GPU equals oracle bit for
    bit.  The last two sheets are critical (det A = 0): kappa = 1 sends every
    ray to beta = 0, a pixel corner of the window, and kappa + gamma1 = 1
    sends every ray to beta_x = 0, a column edge."""
    lens = (kc, g1, g2, [], [], [])
    rays = (-2.0 - 1 / 64, -1.5 - 1 / 128, 1 / 32, 1 / 64, 128, 192, 0, 0)
    pix = (-1.5, -1.25, 1 / 16, 1 / 8, 48, 20)
    ox, oy, ob = ora.shoot(lens, rays, pix)
    with R.Context(lens) as ctx:
        for prec in ("fp64", "fp32_bulk"):
            bx, by, b = ctx.shoot(rays, prec, pix)
            np.testing.assert_array_equal(_np(bx), ox)
            np.testing.assert_array_equal(_np(by), oy)
            np.testing.assert_array_equal(_np(b), ob)


# ----------------------------------------------------------------- small config
@pytest.fixture(scope="module")
def small():
    return W.plain_fp64_small()


@pytest.fixture(scope="module")
def small_oracle(small):
    lens, rays, pix = small.lens.as_tuple(), small.rays.as_tuple(), small.pix.as_tuple()
    bx, by, b = ora.shoot(lens, rays, pix)
    counts, n = ora.map_counts(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    return bx, by, b, counts, n, s


def test_small_config_fp64_per_ray(torch, small, small_oracle):
    bx, by, b, _, _, s = small_oracle
    near = _near_edges(bx, by, s, small.pix.as_tuple())
    with R.Context(small.lens) as ctx:
        for shape in FP64_SHAPES:
            _say("shape", shape)
            _set64(ctx, shape)
            gx, gy, gb = ctx.shoot(small.rays, "fp64", small.pix)
            gx, gy, gb = _np(gx), _np(gy), _np(gb)
            assert np.all(np.abs(gx - bx) <= BETA_TOL * s)
            assert np.all(np.abs(gy - by) <= BETA_TOL * s)
            _assert_bins(gb, b, near, str(shape))


def test_small_config_fp64_map(torch, small, small_oracle):
    bx, by, b, counts, n, s = small_oracle
    n_near = int(_near_edges(bx, by, s, small.pix.as_tuple()).sum())
    with R.Context(small.lens) as ctx:
        maps = []
        for shape in FP64_SHAPES:
            _set64(ctx, shape)
            m, nb = ctx.map(small.rays, small.pix, "fp64", n_binned=True)
            m = _np(m)
            assert nb == m.sum()
            _assert_map(m, counts, n, nb, n_near, str(shape))
            maps.append(m)
        for m in maps[1:]:
            np.testing.assert_array_equal(m, maps[0])


def test_run_to_run_identical(torch, small):
    with R.Context(small.lens) as ctx:
        a = _np(ctx.map(small.rays, small.pix, "fp64"))
        b = _np(ctx.map(small.rays, small.pix, "fp64"))
        np.testing.assert_array_equal(a, b)
        c = ctx.map(small.rays, small.pix, "fp64")
        ctx.map(small.rays, small.pix, "fp64", counts=c)   # accumulates
        np.testing.assert_array_equal(_np(c), 2 * a)


@pytest.mark.parametrize("i0,j0,nx,ny", [(0, 0, 1, 1), (3, 5, 17, 3), (990, 0, 10, 1000),
                                         (0, 999, 1000, 1), (123, 456, 77, 65), (0, 0, 33, 65)])
def test_ragged_blocks(torch, small, small_oracle, i0, j0, nx, ny):
    bx, by, b, _, _, s = small_oracle
    blk = small.rays.block(i0, j0, nx, ny)
    with R.Context(small.lens) as ctx:
        for prec in ("fp64",):
            gx, gy, gb = ctx.shoot(blk, prec, small.pix)
            sl = (slice(j0, j0 + ny), slice(i0, i0 + nx))
            assert np.all(np.abs(_np(gx) - bx[sl]) <= BETA_TOL * s[sl])
            assert np.all(np.abs(_np(gy) - by[sl]) <= BETA_TOL * s[sl])
            np.testing.assert_array_equal(_np(gb), b[sl])


def test_empty_block_is_noop(torch, small):
    with R.Context(small.lens) as ctx:
        counts = torch.zeros((small.pix.NY, small.pix.NX), dtype=torch.int32, device="cuda")
        _, nb = ctx.map(small.rays.block(0, 0, 0, 5), small.pix, "fp64", counts=counts, n_binned=True)
        assert nb == 0 and int(counts.sum()) == 0
        bx, by, b = ctx.shoot(small.rays.block(0, 0, 7, 0), "fp64", small.pix)
        assert bx.numel() == 0


def test_band_additivity(torch, small):
    """map(lattice) = sum of maps of its row bands and column blocks, exactly."""
    with R.Context(small.lens) as ctx:
        full = _np(ctx.map(small.rays, small.pix, "fp64"))
        acc = torch.zeros((small.pix.NY, small.pix.NX), dtype=torch.int32, device="cuda")
        for j0, ny in ((0, 333), (333, 1), (334, 666)):
            for i0, nx in ((0, 500), (500, 500)):
                ctx.map(small.rays.block(i0, j0, nx, ny), small.pix, "fp64", counts=acc)
        np.testing.assert_array_equal(_np(acc), full)


def test_zero_stars_and_massless_star(torch, small):
    """n_stars = 0 is a pure sheet; a massless star changes nothing: in FP64
    (one pass and split), FP32-bulk and the expansion mode."""
    lens0 = (small.lens.kappa_c, small.lens.gamma1, small.lens.gamma2, [], [], [])
    lens1 = (small.lens.kappa_c, small.lens.gamma1, small.lens.gamma2, [0.3], [0.7], [0.0])
    rays = small.rays.block(100, 100, 200, 150)
    ox, oy, ob = ora.shoot(lens0, rays.as_tuple(), small.pix.as_tuple())
    for lens in (lens0, lens1):
        with R.Context(lens) as ctx:
            # every path adds an exact zero to the macro term: the same beta bit for bit
            for prec, split in (("fp64", 1), ("fp64", 4), ("fp32_bulk", 1), ("fp64_expansion", 1)):
                ctx.set_star_split(split)
                gx, gy, gb = ctx.shoot(rays, prec, small.pix)
                np.testing.assert_array_equal(_np(gx), ox, err_msg=f"{prec} split {split}")
                np.testing.assert_array_equal(_np(gy), oy, err_msg=f"{prec} split {split}")
                np.testing.assert_array_equal(_np(gb), ob, err_msg=f"{prec} split {split}")
            ctx.set_star_split(1)
            m = ctx.map(rays, small.pix, "fp64")
            want = np.bincount(ob[ob >= 0], minlength=small.pix.NX * small.pix.NY)
            np.testing.assert_array_equal(_np(m).ravel(), want)


def test_fp32_bulk_small(torch, small, small_oracle):
    _, _, b, _, _, _ = small_oracle
    with R.Context(small.lens) as ctx:
        for shape in FP32_SHAPES:
            ctx.set_tile("fp32_bulk", shape[0], shape[1], star_tile=shape[2])
            _, _, gb = ctx.shoot(small.rays, "fp32_bulk", small.pix)
            frac = np.count_nonzero(_np(gb) != b) / b.size
            _say("fp32 shape", shape, "misbinned", frac)
            assert frac <= MISBIN_FP32


# ----------------------------------------------------------------- large configs
def _sample(rng, nx, ny, n):
    return rng.integers(0, nx, n), rng.integers(0, ny, n)


def test_large_config_full_size(torch):
    """8192^2 rays, 16384 stars, the launch the benchmark times: the map equals
    the histogram of the per-ray bins, and sampled rays match the oracle."""
    w = W.plain_fp64_large()
    rng = np.random.default_rng(0)
    ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 1500)
    ox, oy, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
    tx, ty = ora.image_angles(w.rays.as_tuple())
    s = ora.error_scale(w.lens.as_tuple(), tx[ii], ty[jj])
    near = _near_edges(ox, oy, s, w.pix.as_tuple())
    with R.Context(w.lens) as ctx:
        _say("map fp64")
        m, nb = ctx.map(w.rays, w.pix, "fp64", n_binned=True)
        _say("shoot fp64")
        gx, gy, gb = ctx.shoot(w.rays, "fp64", w.pix)
        hist = torch.bincount(gb[gb >= 0].long(), minlength=w.pix.NX * w.pix.NY)
        assert torch.equal(hist.to(torch.int32).view(w.pix.NY, w.pix.NX), m)
        assert nb == int((gb >= 0).sum())
        jt, it = torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")
        _assert_bins(_np(gb[jt, it]), ob, near, "sampled rays")
        assert np.all(np.abs(_np(gx[jt, it]) - ox) <= BETA_TOL * s)
        assert np.all(np.abs(_np(gy[jt, it]) - oy) <= BETA_TOL * s)
        del gx, gy
        _say("fp32 bulk")
        _, _, fb = ctx.shoot(w.rays, "fp32_bulk", w.pix)
        frac = float((fb != gb).sum()) / gb.numel()
        _say("large config fp32-bulk misbinned fraction", frac)
        assert frac <= MISBIN_FP32
        mean_mu = nb * w.rays.dx * w.rays.dy / (20.0 * 20.0)
        _say("mean magnification", mean_mu, "sheet", W.mean_magnification(0.45, 0.35, 0.1))


def test_precision_study_subtile(torch):
    """262144 stars: FP32-bulk against FP64 on the central 2048^2 rays."""
    w = W.precision_study()
    sub = W.precision_subtile(w, 2048)
    rng = np.random.default_rng(1)
    ii, jj = _sample(rng, sub.nx, sub.ny, 64)
    _, _, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(),
                              ii + sub.i0, jj + sub.j0)
    with R.Context(w.lens) as ctx:
        _say("fp64 subtile")
        _, _, b64 = ctx.shoot(sub, "fp64", w.pix, beta=False)
        _say("fp32 subtile")
        _, _, b32 = ctx.shoot(sub, "fp32_bulk", w.pix, beta=False)
        sel = _np(b64[torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")])
        assert np.count_nonzero(sel != ob) == 0
        frac = float((b32 != b64).sum()) / b64.numel()
        _say("precision-study fp32-bulk misbinned fraction", frac)
        assert frac <= MISBIN_FP32


# ----------------------------------------------------------------- batch
@pytest.fixture(scope="module")
def small_batch():
    return W.batch_workloads(n_sets=9, rays_per_side=700, npix=128, n_lo=50, n_hi=3000,
                             seed=W.BASE_SEED + 77)


def test_batch_equals_single(torch, small_batch):
    ctxs = [R.Context(w.lens) for w in small_batch]
    try:
        for prec in ("fp64", "fp32_bulk"):
            singles = [_np(c.map(w.rays, w.pix, prec)) for c, w in zip(ctxs, small_batch)]
            maps = R.map_batch(ctxs, [w.rays for w in small_batch], [w.pix for w in small_batch], prec)
            for s, m in zip(singles, maps):
                np.testing.assert_array_equal(_np(m), s)
    finally:
        for c in ctxs:
            c.close()


def test_batch_graph_replays(torch, small_batch):
    """The captured launch is replayed on later calls; every replay adds the
    same counts, with other GPU work in between."""
    ctxs = [R.Context(w.lens) for w in small_batch]
    try:
        rays = [w.rays for w in small_batch]
        pix = [w.pix for w in small_batch]
        want = [_np(c.map(w.rays, w.pix, "fp64")) for c, w in zip(ctxs, small_batch)]
        maps = [torch.zeros((p.NY, p.NX), dtype=torch.int32, device="cuda") for p in pix]
        for rep in range(1, 5):
            R.map_batch(ctxs, rays, pix, "fp64", counts=maps)
            junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
            torch.cuda.synchronize()
            for m, wnt in zip(maps, want):
                np.testing.assert_array_equal(_np(m), rep * wnt)
            del junk
    finally:
        for c in ctxs:
            c.close()


def test_batch_with_empty_and_ragged_sets(torch, small_batch):
    ctxs = [R.Context(w.lens) for w in small_batch[:3]]
    try:
        rays = [small_batch[0].rays.block(0, 0, 0, 10), small_batch[1].rays.block(5, 7, 33, 17),
                small_batch[2].rays]
        pix = [w.pix for w in small_batch[:3]]
        maps = R.map_batch(ctxs, rays, pix, "fp64")
        for c, r, p, m in zip(ctxs, rays, pix, maps):
            np.testing.assert_array_equal(_np(m), _np(c.map(r, p, "fp64")))
    finally:
        for c in ctxs:
            c.close()


def test_batch_with_starless_and_one_star_sets(torch, small_batch):
    """Sets of 0, 1 and 2 stars beside a full one in one batch: in both
    precisions each set's map equals its single-launch map, and the FP64
    maps of the small sets equal the oracle's (up to rays within the beta
    bar of a pixel edge)."""
    w = small_batch[0]
    lenses = [(0.1, 0.2, 0.0, [], [], []),
              (0.0, 0.3, -0.1, [0.21], [-0.37], [0.8]),
              (0.2, -0.1, 0.05, [0.5, -1.1], [0.3, 0.9], [0.4, 1.0]),
              w.lens.as_tuple()]
    ctxs = [R.Context(l) for l in lenses]
    try:
        rays, pix = [w.rays] * len(lenses), [w.pix] * len(lenses)
        for prec in ("fp64", "fp32_bulk"):
            maps = R.map_batch(ctxs, rays, pix, prec)
            for k, (c, m) in enumerate(zip(ctxs, maps)):
                np.testing.assert_array_equal(_np(m), _np(c.map(w.rays, w.pix, prec)), err_msg=f"{prec} set {k}")
        maps = R.map_batch(ctxs, rays, pix, "fp64")
        threads = max(1, min(16, os.cpu_count() or 1))
        for k in range(3):
            ox, oy, ob, sc = _oracle_threaded(lenses[k], w.rays, w.pix.as_tuple(), threads)
            want = np.bincount(ob[ob >= 0].ravel(), minlength=w.pix.NX * w.pix.NY).reshape(w.pix.NY, w.pix.NX)
            n_near = int(_near_edges(ox, oy, sc, w.pix.as_tuple()).sum())
            g = _np(maps[k])
            _assert_map(g, want, int((ob >= 0).sum()), int(g.sum()), n_near, f"set {k} against the oracle")
    finally:
        for c in ctxs:
            c.close()


def test_batch_matches_oracle(torch, small_batch):
    """Every set's batched map against the oracle's map of that set (the
    oracle's per-ray bins on host threads): FP64 equal up to the rays near
    pixel edges, FP32-bulk within 1e-4 misbinned rays per set."""
    threads = max(1, min(16, os.cpu_count() or 1))
    ctxs = [R.Context(w.lens) for w in small_batch]
    try:
        rays, pix = [w.rays for w in small_batch], [w.pix for w in small_batch]
        m64 = R.map_batch(ctxs, rays, pix, "fp64")
        m32 = R.map_batch(ctxs, rays, pix, "fp32_bulk")
        for k, w in enumerate(small_batch):
            ox, oy, ob, s = _oracle_threaded(w.lens.as_tuple(), w.rays, w.pix.as_tuple(), threads)
            counts = np.bincount(ob[ob >= 0].ravel(), minlength=w.pix.NX * w.pix.NY).reshape(w.pix.NY, w.pix.NX)
            n = int((ob >= 0).sum())
            n_near = int(_near_edges(ox, oy, s, w.pix.as_tuple()).sum())
            g64 = _np(m64[k])
            _assert_map(g64, counts, n, int(g64.sum()), n_near, f"set {k} fp64")
            g32 = _np(m32[k])
            frac = 0.5 * (np.abs(g32.astype(np.int64) - counts).sum() + abs(int(g32.sum()) - n)) / ob.size
            _say(f"set {k}: {w.lens.n_stars} stars, fp64 near edges {n_near}, fp32-bulk misbinned >= {frac:.2e}")
            assert frac <= MISBIN_FP32, k
    finally:
        for c in ctxs:
            c.close()


def _on_star_lens(rng):
    """Stars exactly on lattice points of the dyadic lattice of
    test_star_on_a_ray_drops_only_that_ray, plus stars elsewhere."""
    x0, y0, d = -1.5, -1.25, 1.0 / 32
    on = [(5, 7), (40, 30), (77, 63), (0, 0), (95, 79), (50, 12), (17, 23)]
    xs = [x0 + (i + 0.5) * d for i, _ in on] + list(rng.uniform(-2.0, 2.0, 20))
    ys = [y0 + (j + 0.5) * d for _, j in on] + list(rng.uniform(-2.0, 2.0, 20))
    ms = list(rng.uniform(0.01, 0.05, len(xs)))
    rays = (x0, y0, d, d, 96, 80, 0, 0)
    return (0.05, 0.1, -0.03, np.array(xs), np.array(ys), np.array(ms)), rays, on


@pytest.mark.parametrize("parts", [1, 3])
def test_star_on_a_ray_drops_only_that_ray(torch, parts):
    """Stars exactly on lattice points, whose neighbours in the lane's
    reciprocal groups (columns i + 16 a, rows j + 16 b) lie inside the
    block: for every FP64 shape, one pass and split, only the rays on stars
    are dropped, and every other ray matches the oracle."""
    rng = np.random.default_rng(40)
    lens, rays, on = _on_star_lens(rng)
    pix = (-2.0, -2.0, 4 / 64, 4 / 64, 64, 64)
    ox, oy, ob = ora.shoot(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    fin = np.isfinite(ox) & np.isfinite(oy)
    assert np.count_nonzero(~fin) == len(on)
    assert all(not fin[j, i] for i, j in on)
    near = _near_edges(ox, oy, s, pix)
    counts = np.bincount(ob[ob >= 0].ravel(), minlength=64 * 64).reshape(64, 64)
    with R.Context(lens) as ctx:
        ctx.set_star_split(parts)
        for shape in FP64_SHAPES:
            _set64(ctx, shape)
            gx, gy, gb = (_np(t) for t in ctx.shoot(rays, "fp64", pix))
            gfin = np.isfinite(gx) & np.isfinite(gy)
            assert np.array_equal(gfin, fin), (shape, np.argwhere(gfin != fin)[:4])
            assert np.all(np.abs(gx[fin] - ox[fin]) <= BETA_TOL * s[fin]), shape
            assert np.all(np.abs(gy[fin] - oy[fin]) <= BETA_TOL * s[fin]), shape
            _assert_bins(gb, ob, near, str(shape))
            m, nb = ctx.map(rays, pix, "fp64", n_binned=True)
            _assert_map(_np(m), counts, int((ob >= 0).sum()), nb, int(near.sum()), str(shape))


FP32_BETA_TOL = 1e-5   # FP32-bulk: ~30 FP32 terms of relative error < 1e-6 each, partial sums in FP64


def test_star_on_a_ray_fp32_bulk(torch):
    """FP32-bulk with stars exactly on lattice points: only the rays on
    stars are dropped; every other ray's beta is within 1e-5 S of the
    oracle's and, away from pixel edges by more than that, in its pixel."""
    rng = np.random.default_rng(42)
    lens, rays, on = _on_star_lens(rng)
    pix = (-2.0, -2.0, 4 / 64, 4 / 64, 64, 64)
    ox, oy, ob = ora.shoot(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    fin = np.isfinite(ox) & np.isfinite(oy)
    assert np.count_nonzero(~fin) == len(on)
    X0, Y0, Px, Py = pix[:4]
    with np.errstate(invalid="ignore"):
        du = np.abs((ox - X0) / Px - np.round((ox - X0) / Px)) * Px
        dv = np.abs((oy - Y0) / Py - np.round((oy - Y0) / Py)) * Py
    band = fin & ((du <= FP32_BETA_TOL * s) | (dv <= FP32_BETA_TOL * s))
    with R.Context(lens) as ctx:
        for shape in FP32_SHAPES:
            ctx.set_tile("fp32_bulk", shape[0], shape[1], star_tile=shape[2])
            gx, gy, gb = (_np(t) for t in ctx.shoot(rays, "fp32_bulk", pix))
            assert np.array_equal(np.isfinite(gx) & np.isfinite(gy), fin), shape
            assert np.all(np.abs(gx[fin] - ox[fin]) <= FP32_BETA_TOL * s[fin]), shape
            assert np.all(np.abs(gy[fin] - oy[fin]) <= FP32_BETA_TOL * s[fin]), shape
            assert np.count_nonzero((gb != ob) & ~band) == 0, shape


def test_star_on_a_ray_in_a_batch(torch):
    """The same lens in a batch, beside another set, for every FP64 shape:
    its batched map equals the oracle's."""
    rng = np.random.default_rng(41)
    lens, rays, _ = _on_star_lens(rng)
    pix = (-2.0, -2.0, 4 / 64, 4 / 64, 64, 64)
    ox, oy, ob = ora.shoot(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    counts = np.bincount(ob[ob >= 0].ravel(), minlength=64 * 64).reshape(64, 64)
    n_near = int(_near_edges(ox, oy, s, pix).sum())
    other = (0.1, 0.0, 0.0, rng.uniform(-2, 2, 50), rng.uniform(-2, 2, 50), rng.uniform(0.01, 0.1, 50))
    ctxs = [R.Context(lens), R.Context(other)]
    try:
        for shape in FP64_SHAPES:
            for c in ctxs:
                _set64(c, shape)
            maps = R.map_batch(ctxs, [rays, rays], [pix, pix], "fp64")
            g = _np(maps[0])
            _assert_map(g, counts, int((ob >= 0).sum()), int(g.sum()), n_near, str(shape))
    finally:
        for c in ctxs:
            c.close()


# ----------------------------------------------------------------- errors on the device
def test_device_pointer_errors(torch, small):
    with R.Context(small.lens) as ctx:
        host = np.zeros((small.pix.NY, small.pix.NX), np.int32)
        lib = R.load()
        r = R.rays_struct(small.rays)
        p = R.pixels_struct(small.pix)
        code = lib.raysh_map(ctx.handle, r, p, 0, host.ctypes.data, None)
        assert code == R.EINVAL and "device memory" in lib.raysh_last_error().decode()
        big = R.Pixels(-5.0, -5.0, 0.001, 0.001, 10000, 10000)   # 400 MB map
        tiny = torch.zeros(16, dtype=torch.int32, device="cuda")
        code = lib.raysh_map(ctx.handle, r, big, 0, tiny.data_ptr(), None)
        assert code == R.EINVAL and "needed" in lib.raysh_last_error().decode()
        assert int(tiny.abs().sum()) == 0
        with pytest.raises(R.RayshError):
            ctx.set_tile("fp64", 3, 3, share=2)


# ----------------------------------------------------------------- autotuner
def test_autotune_picks_compiled_shape_and_caches(torch, small, tmp_path):
    cache = str(tmp_path / "tune.txt")
    with R.Context(small.lens) as ctx:
        ref = _np(ctx.map(small.rays, small.pix, "fp64"))
        t64 = ctx.autotune(small.rays, small.pix, "fp64", cache_path=cache)
        assert tuple(t64) in FP64_SHAPES and ctx.get_tile("fp64") == t64
        np.testing.assert_array_equal(_np(ctx.map(small.rays, small.pix, "fp64")), ref)
        t32 = ctx.autotune(small.rays, small.pix, "fp32_bulk", cache_path=cache)
        assert (t32[0], t32[1], t32[3]) in FP32_SHAPES
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == 2
    with R.Context(small.lens) as ctx:   # a cache hit gives the same choice without timing
        assert ctx.autotune(small.rays, small.pix, "fp64", cache_path=cache) == t64
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 2


def test_autotune_batch_picks_compiled_shape_and_caches(torch, small_batch, tmp_path):
    """raysh_autotune_batch times the shapes with the batch kernel, sets the
    fastest in every context, and the batch then equals its single launches
    with that shape; a second call is answered from the cache."""
    cache = str(tmp_path / "tune_batch.txt")
    ctxs = [R.Context(w.lens) for w in small_batch]
    try:
        rays, pix = [w.rays for w in small_batch], [w.pix for w in small_batch]
        t64 = R.autotune_batch(ctxs, rays, pix, "fp64", cache_path=cache)
        assert tuple(t64) in FP64_SHAPES and all(c.get_tile("fp64") == t64 for c in ctxs)
        maps = R.map_batch(ctxs, rays, pix, "fp64")
        for c, w, m in zip(ctxs, small_batch, maps):
            assert torch.equal(m, c.map(w.rays, w.pix, "fp64"))
        t32 = R.autotune_batch(ctxs, rays, pix, "fp32_bulk", cache_path=cache)
        assert (t32[0], t32[1], t32[3]) in FP32_SHAPES and t32[2] == 0
        lines = [l for l in open(cache).read().split("\n") if l.strip()]
        assert len(lines) == 2 and all(" batch " in l for l in lines)
        for c in ctxs:
            c.set_tile("fp64", 2, 2, share=2)
        assert R.autotune_batch(ctxs, rays, pix, "fp64", cache_path=cache) == t64   # a cache hit
        assert all(c.get_tile("fp64") == t64 for c in ctxs)
        assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 2
    finally:
        for c in ctxs:
            c.close()


# ----------------------------------------------------------------- full sizes, maximum sizes
def test_batch_full_size_equals_single_launches(torch):
    """The 64-set workload at full size (4096^2 rays per set, N* 511..43689):
    every set's batched map equals its single-launch map exactly, in both
    precisions, and sampled rays of the largest and smallest sets match the
    oracle."""
    sets = W.batch_workloads()
    ctxs = [R.Context(w.lens) for w in sets]
    try:
        rays, pix = [w.rays for w in sets], [w.pix for w in sets]
        for prec in ("fp64", "fp32_bulk"):
            _say("batch", prec)
            maps = R.map_batch(ctxs, rays, pix, prec)
            for c, w, m in zip(ctxs, sets, maps):
                assert torch.equal(m, c.map(w.rays, w.pix, prec))
        rng = np.random.default_rng(3)
        order = np.argsort([w.lens.n_stars for w in sets])
        for s in (order[0], order[-1]):
            w = sets[s]
            ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 200)
            _, _, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
            _, _, gb = ctxs[s].shoot(w.rays, "fp64", w.pix, beta=False)
            sel = _np(gb[torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")])
            assert np.count_nonzero(sel != ob) == 0
    finally:
        for c in ctxs:
            c.close()


def test_precision_study_full_lattice(torch):
    """16384^2 rays x 262144 stars (7e13 interactions): sampled rays of the
    whole lattice match the oracle, the map equals the histogram of the bins,
    and the FP32-bulk form stays within 1e-4 misbinned rays."""
    w = W.precision_study()
    rng = np.random.default_rng(4)
    ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 48)
    _, _, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
    with R.Context(w.lens) as ctx:
        _say("full lattice fp64 map")
        m = ctx.map(w.rays, w.pix, "fp64")
        _say("full lattice fp64 bins")
        _, _, b64 = ctx.shoot(w.rays, "fp64", w.pix, beta=False)
        hist = torch.bincount(b64[b64 >= 0].long(), minlength=w.pix.NX * w.pix.NY)
        assert torch.equal(hist.to(torch.int32).view(w.pix.NY, w.pix.NX), m)
        sel = _np(b64[torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")])
        assert np.count_nonzero(sel != ob) == 0
        _say("full lattice fp32 bins")
        _, _, b32 = ctx.shoot(w.rays, "fp32_bulk", w.pix, beta=False)
        frac = float((b32 != b64).sum()) / b64.numel()
        _say("full precision-study lattice fp32-bulk misbinned fraction", frac)
        assert frac <= MISBIN_FP32


def test_maximum_sizes(torch):
    """A map of 46340^2 = 2147395600 pixels (just under 2^31) and a call of
    46340^2 rays (dyadic sheet, exact): the int32 pixel index and the 64-bit
    ray offsets hold at the limits, and the largest call is still accepted."""
    n = 46340
    P = 1.0 / 4096
    pix = (-n * P / 2, -n * P / 2, P, P, n, n)
    # identity lens: ray (i, j) sits at the centre of pixel (i, j)
    lens = (0.0, 0.0, 0.0, [], [], [])
    rays = (-n * P / 2, -n * P / 2, P, P, n, n, 0, 0)
    with R.Context(lens) as ctx:
        counts, nb = ctx.map(rays, pix, "fp64", n_binned=True)
        assert nb == n * n
        assert int(counts.min()) == 1 and int(counts.max()) == 1
        del counts
        # the last rows: bins equal their own linear index
        blk = (rays[0], rays[1], P, P, n, 3, 0, n - 3)
        _, _, b = ctx.shoot(blk, "fp64", pix, beta=False)
        want = torch.arange((n - 3) * n, n * n, device="cuda", dtype=torch.int64).view(3, n)
        assert torch.equal(b.long(), want)
    bad = R.Rays(0.0, 0.0, 1.0, 1.0, 46341, 46341, 0, 0)   # 2147488281 rays > 2^31 - 1
    lib = R.load()
    assert lib.raysh_shoot(None, bad, 0, None, None, None, None) == R.EOVERFLOW


# ----------------------------------------------------------------- split star sum (many stars, few rays)
@pytest.mark.parametrize("parts", [2, 3, 7, 40])
def test_star_split_matches_oracle(torch, small, small_oracle, parts):
    """Each ray's star sum split over `parts` star ranges (40 > 100/4 groups:
    some ranges are empty) still matches the oracle ray by ray."""
    bx, by, b, counts, n, s = small_oracle
    near = _near_edges(bx, by, s, small.pix.as_tuple())
    with R.Context(small.lens) as ctx:
        ctx.set_star_split(parts)
        gx, gy, gb = ctx.shoot(small.rays, "fp64", small.pix)
        assert np.all(np.abs(_np(gx) - bx) <= BETA_TOL * s)
        assert np.all(np.abs(_np(gy) - by) <= BETA_TOL * s)
        n_near = _assert_bins(_np(gb), b, near, f"{parts} parts")
        m, nb = ctx.map(small.rays, small.pix, "fp64", n_binned=True)
        _assert_map(_np(m), counts, n, nb, n_near, f"{parts} parts")
        # band additivity holds exactly at a fixed part count
        acc = torch.zeros_like(m)
        for j0, ny in ((0, 400), (400, 600)):
            ctx.map(small.rays.block(0, j0, 1000, ny), small.pix, "fp64", counts=acc)
        assert torch.equal(acc, m)


def test_star_split_edge_cases(torch):
    """Star counts that are not a multiple of the group size, a single star,
    no stars, and ragged blocks, with splits."""
    rng = np.random.default_rng(8)
    pix = (-2.0, -2.0, 4 / 64, 4 / 64, 64, 64)
    rays = (-3.0, -2.5, 6 / 77, 5 / 53, 77, 53, 0, 0)
    for n_st in (0, 1, 5, 131):
        xs, ys = rng.uniform(-2, 2, n_st), rng.uniform(-2, 2, n_st)
        ms = rng.uniform(0.1, 1, n_st)
        lens = (0.1, 0.2, -0.05, xs, ys, ms)
        ox, oy, ob = ora.shoot(lens, rays, pix)
        s = ora.error_scale_block(lens, rays)
        near = _near_edges(ox, oy, s, pix)
        with R.Context(lens) as ctx:
            for parts in (0, 2, 9):
                ctx.set_star_split(parts)
                gx, gy, gb = ctx.shoot(rays, "fp64", pix)
                assert np.all(np.abs(_np(gx) - ox) <= BETA_TOL * s), (n_st, parts)
                assert np.all(np.abs(_np(gy) - oy) <= BETA_TOL * s), (n_st, parts)
                _assert_bins(_np(gb), ob, near, f"{n_st} stars, {parts} parts")
        with pytest.raises(R.RayshError):
            R.Context(lens).set_star_split(-1)


def test_large_star_field_split(torch):
    """4194304 stars, 256^2 rays: the automatic split fills the GPU; sampled
    rays match the oracle; the map equals the histogram of the bins."""
    w = W.large_star_field(1 << 22, 256, 256)
    rng = np.random.default_rng(9)
    ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 12)
    ox, oy, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
    tx, ty = ora.image_angles(w.rays.as_tuple())
    s = ora.error_scale(w.lens.as_tuple(), tx[ii], ty[jj])
    near = _near_edges(ox, oy, s, w.pix.as_tuple())
    with R.Context(w.lens) as ctx:
        ctx.set_star_split(0)
        gx, gy, gb = ctx.shoot(w.rays, "fp64", w.pix)
        m = ctx.map(w.rays, w.pix, "fp64")
        hist = torch.bincount(gb[gb >= 0].long(), minlength=w.pix.NX * w.pix.NY)
        assert torch.equal(hist.to(torch.int32).view(w.pix.NY, w.pix.NX), m)
        jt, it = torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")
        _assert_bins(_np(gb[jt, it]), ob, near, "sampled rays")
        assert np.all(np.abs(_np(gx[jt, it]) - ox) <= BETA_TOL * s)
        assert np.all(np.abs(_np(gy[jt, it]) - oy) <= BETA_TOL * s)


def test_star_field_of_2_28_stars_split(torch):
    """The regime of Sec. 4 (very many stars, few rays): 2^28 stars resident
    on the GPU (8 GiB of 32-byte records) x 256^2 rays, the star sum split
    automatically over workgroups.  8 sampled rays match the oracle within
    the FP64 bar, and the map equals the histogram of the per-ray bins."""
    n = 1 << 28
    _say("drawing 2^28 stars")
    w = W.large_star_field(n, 256, 256)
    rng = np.random.default_rng(28)
    ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 8)
    with R.Context(w.lens) as ctx:
        assert R.load().raysh_n_stars(ctx.handle) == n
        ctx.set_star_split(0)
        _say("gpu: split star sum")
        gx, gy, gb = ctx.shoot(w.rays, "fp64", w.pix)
        m = ctx.map(w.rays, w.pix, "fp64")
        hist = torch.bincount(gb[gb >= 0].long(), minlength=w.pix.NX * w.pix.NY)
        assert torch.equal(hist.to(torch.int32).view(w.pix.NY, w.pix.NX), m)
        jt, it = torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")
        gx, gy, gb = _np(gx[jt, it]), _np(gy[jt, it]), _np(gb[jt, it])
    _say("oracle: 8 rays x 2^28 stars")
    ox, oy, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
    tx, ty = ora.image_angles(w.rays.as_tuple())
    s = ora.error_scale(w.lens.as_tuple(), tx[ii], ty[jj])
    _say("max |dbeta|/S", float(np.max(np.maximum(np.abs(gx - ox), np.abs(gy - oy)) / s)))
    assert np.all(np.abs(gx - ox) <= BETA_TOL * s)
    assert np.all(np.abs(gy - oy) <= BETA_TOL * s)
    _assert_bins(gb, ob, _near_edges(ox, oy, s, w.pix.as_tuple()), "2^28 stars")


# ----------------------------------------------------------------- far-field expansion
@pytest.mark.parametrize("block", [1, 2, 4])
def test_expansion_matches_oracle_small(torch, small, small_oracle, block):
    """RAYSH_FP64_EXPANSION holds the FP64 bar ray by ray on the 100-star
    workload (a few far stars per tile), for several far criteria and each
    workgroup block (1, 2 or 4 tiles per side; 1000^2 rays are 16 x 16
    tiles, the last row and column ragged)."""
    bx, by, b, counts, n, s = small_oracle
    near = _near_edges(bx, by, s, small.pix.as_tuple())
    with R.Context(small.lens) as ctx:
        ctx.set_expansion_block(block)
        for cells in ("never", "always"):
            ctx.set_expansion_cells(cells)
            for theta in (0.3, 0.25, 0.1):
                ctx.set_expansion(theta)
                gx, gy, gb = ctx.shoot(small.rays, "fp64_expansion", small.pix)
                assert np.all(np.abs(_np(gx) - bx) <= BETA_TOL * s), (cells, theta)
                assert np.all(np.abs(_np(gy) - by) <= BETA_TOL * s), (cells, theta)
                n_near = _assert_bins(_np(gb), b, near, f"cells {cells}, theta {theta}")
        m, nb = ctx.map(small.rays, small.pix, "fp64_expansion", n_binned=True)
        _assert_map(_np(m), counts, n, nb, n_near, "expansion map")
        with pytest.raises(R.RayshError):
            ctx.set_expansion(0.0)
        with pytest.raises(R.RayshError):
            ctx.set_expansion(0.5)
        with pytest.raises(R.RayshError):
            ctx.set_expansion_block(3)
        with pytest.raises(R.RayshError):
            R.check(R.load().raysh_set_expansion_cells(ctx.handle, 3))
        with pytest.raises(R.RayshError):
            ctx.set_tile("fp64_expansion", 4, 4)
        with pytest.raises(R.RayshError):
            R.map_batch([ctx], [small.rays], [small.pix], "fp64_expansion")


def test_expansion_workspace_grows_in_one_context(torch, small, small_oracle):
    """One context maps lattice blocks of growing size, and changes its
    workgroup block, in the expansion mode: the workspace of the blocks'
    coefficients and near lists is reallocated as needed, and every call
    still matches the oracle ray by ray."""
    bx, by, b, _, _, s = small_oracle
    near_all = _near_edges(bx, by, s, small.pix.as_tuple())
    nx_all = small.rays.nx
    with R.Context(small.lens) as ctx:
        for block, (nx, ny) in ((1, (64, 64)), (1, (300, 200)), (4, (300, 200)), (1, (1000, 1000)),
                                (2, (130, 70))):
            ctx.set_expansion_block(block)
            sub = small.rays.block(0, 0, nx, ny)
            gx, gy, gb = ctx.shoot(sub, "fp64_expansion", small.pix)
            sel = (slice(0, ny), slice(0, nx))
            want_x = bx.reshape(-1, nx_all)[sel].ravel()
            want_y = by.reshape(-1, nx_all)[sel].ravel()
            want_b = b.reshape(-1, nx_all)[sel].ravel()
            scale = s.reshape(-1, nx_all)[sel].ravel()
            assert np.all(np.abs(_np(gx).ravel() - want_x) <= BETA_TOL * scale), (block, nx, ny)
            assert np.all(np.abs(_np(gy).ravel() - want_y) <= BETA_TOL * scale), (block, nx, ny)
            _assert_bins(_np(gb), want_b, near_all.reshape(-1, nx_all)[sel], f"block {block}, {nx}x{ny}")


@pytest.mark.parametrize("block", [2, 4])
@pytest.mark.parametrize("i0,j0,nx,ny", [(0, 0, 300, 200), (37, 501, 130, 499), (999, 0, 1, 1000),
                                         (5, 5, 64, 64), (0, 0, 0, 10)])
def test_expansion_ragged_blocks(torch, small, small_oracle, block, i0, j0, nx, ny):
    """Lattice blocks that fill a workgroup's tiles partly (or not at all)."""
    bx, by, b, _, _, s = small_oracle
    blk = small.rays.block(i0, j0, nx, ny)
    with R.Context(small.lens) as ctx:
        ctx.set_expansion_block(block)
        gx, gy, gb = ctx.shoot(blk, "fp64_expansion", small.pix)
        if nx * ny == 0:
            return
        sl = (slice(j0, j0 + ny), slice(i0, i0 + nx))
        assert np.all(np.abs(_np(gx) - bx[sl]) <= BETA_TOL * s[sl])
        assert np.all(np.abs(_np(gy) - by[sl]) <= BETA_TOL * s[sl])
        _assert_bins(_np(gb), b[sl], _near_edges(bx[sl], by[sl], s[sl], small.pix.as_tuple()))


def test_expansion_large_config(torch):
    """16384 stars, 8192^2 rays: sampled rays match the oracle within the
    FP64 bar, and the map differs from the one-pass FP64 map in at most 1e-6
    of the rays."""
    w = W.plain_fp64_large()
    rng = np.random.default_rng(21)
    ii, jj = _sample(rng, w.rays.nx, w.rays.ny, 600)
    ox, oy, ob = ora.shoot_list(w.lens.as_tuple(), w.rays.as_tuple(), w.pix.as_tuple(), ii, jj)
    tx, ty = ora.image_angles(w.rays.as_tuple())
    s = ora.error_scale(w.lens.as_tuple(), tx[ii], ty[jj])
    with R.Context(w.lens) as ctx:
        gx, gy, gb = ctx.shoot(w.rays, "fp64_expansion", w.pix)
        jt, it = torch.as_tensor(jj, device="cuda"), torch.as_tensor(ii, device="cuda")
        assert np.all(np.abs(_np(gx[jt, it]) - ox) <= BETA_TOL * s)
        assert np.all(np.abs(_np(gy[jt, it]) - oy) <= BETA_TOL * s)
        _assert_bins(_np(gb[jt, it]), ob, _near_edges(ox, oy, s, w.pix.as_tuple()), "sampled rays")
        del gx, gy
        _, _, b64 = ctx.shoot(w.rays, "fp64", w.pix, beta=False)
        frac = float((gb != b64).sum()) / gb.numel()
        _say("expansion vs one-pass FP64 misbinned fraction (large config)", frac)
        assert frac <= MISBIN_FP64
        m = ctx.map(w.rays, w.pix, "fp64_expansion")
        hist = torch.bincount(gb[gb >= 0].long(), minlength=w.pix.NX * w.pix.NY)
        assert torch.equal(hist.to(torch.int32).view(w.pix.NY, w.pix.NX), m)


def test_expansion_precision_study_full_lattice(torch):
    """262144 stars, the whole 16384^2 lattice: the expansion's bins differ
    from one-pass FP64 in at most 1e-6 of the rays."""
    w = W.precision_study()
    with R.Context(w.lens) as ctx:
        _, _, be = ctx.shoot(w.rays, "fp64_expansion", w.pix, beta=False)
        _, _, b64 = ctx.shoot(w.rays, "fp64", w.pix, beta=False)
        frac = float((be != b64).sum()) / be.numel()
        _say("expansion vs one-pass FP64 misbinned fraction (precision study)", frac)
        assert frac <= MISBIN_FP64


@pytest.mark.parametrize("cells", ["never", "always"])
@pytest.mark.parametrize("block", [1, 2, 4])
def test_expansion_dense_cluster_falls_back(torch, block, cells):
    """More near stars than the lists hold (3000 stars within 0.3 of the
    lattice centre): those blocks sum every star directly; the result still
    matches the oracle ray by ray.  With a cluster off to one side, other
    blocks of the same lattice take the expansion path."""
    rng = np.random.default_rng(22)
    r = 0.3 * np.sqrt(rng.random(3000))
    phi = 2 * np.pi * rng.random(3000)
    far_r = 20 + 10 * rng.random(500)
    far_p = 2 * np.pi * rng.random(500)
    for shift in (0.0, 1.6):
        xs = np.concatenate([r * np.cos(phi) + shift, far_r * np.cos(far_p)])
        ys = np.concatenate([r * np.sin(phi), far_r * np.sin(far_p)])
        ms = rng.uniform(0.001, 0.002, 3500)
        lens = (0.1, 0.1, 0.0, xs, ys, ms)
        rays = (-2.0, -2.0, 4 / 512, 4 / 512, 512, 512, 0, 0)
        pix = (-1.0, -1.0, 2 / 64, 2 / 64, 64, 64)
        ox, oy, ob = ora.shoot(lens, rays, pix)
        s = ora.error_scale_block(lens, rays)
        with R.Context(lens) as ctx:
            ctx.set_expansion_block(block)
            ctx.set_expansion_cells(cells)
            gx, gy, gb = ctx.shoot(rays, "fp64_expansion", pix)
            assert np.all(np.abs(_np(gx) - ox) <= BETA_TOL * s), shift
            assert np.all(np.abs(_np(gy) - oy) <= BETA_TOL * s), shift
            _assert_bins(_np(gb), ob, _near_edges(ox, oy, s, pix), f"shift {shift}")


@pytest.mark.parametrize("n_stars", [(1 << 19) - 1, 1 << 19, (1 << 19) + 1, 3 * (1 << 19) + 7])
def test_star_upload_chunk_boundaries(torch, n_stars):
    """Star fields around and across the upload's staging chunks (2^19
    records): every star reaches the device (8 x 8 rays against the oracle)."""
    rng = np.random.default_rng(n_stars)
    xs, ys = rng.uniform(-300, 300, n_stars), rng.uniform(-300, 300, n_stars)
    ms = rng.uniform(0.1, 1.0, n_stars)
    lens = (0.05, 0.1, 0.02, xs, ys, ms)
    rays = (-0.5, -0.5, 1 / 8, 1 / 8, 8, 8, 0, 0)
    pix = (-2.0, -2.0, 0.25, 0.25, 16, 16)
    ox, oy, ob = ora.shoot(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    with R.Context(lens) as ctx:
        assert R.load().raysh_n_stars(ctx.handle) == n_stars
        gx, gy, gb = ctx.shoot(rays, "fp64", pix)
        assert np.all(np.abs(_np(gx) - ox) <= BETA_TOL * s)
        assert np.all(np.abs(_np(gy) - oy) <= BETA_TOL * s)
        _assert_bins(_np(gb), ob, _near_edges(ox, oy, s, pix))


@pytest.mark.parametrize("cells", ["never", "always"])
@pytest.mark.parametrize("block", [1, 4])
def test_expansion_degenerate_star_fields(torch, block, cells):
    """No stars, one star, massless stars, a star exactly on a ray (that ray
    is dropped, as in the oracle), stars on a line (a grid of one cell row)
    and stars all at one point (no grid), in the expansion mode."""
    rays = (-1.5, -1.25, 3 / 160, 2.5 / 130, 160, 130, 0, 0)
    pix = (-2.0, -2.0, 4 / 64, 4 / 64, 64, 64)
    tx0 = -1.5 + (37 + 0.5) * (3 / 160)   # the image angle of ray (37, 51)
    ty0 = -1.25 + (51 + 0.5) * (2.5 / 130)
    line = np.linspace(-40.0, 40.0, 400)
    cases = [([], [], []), ([0.3], [-0.2], [1.0]), ([0.3, -0.4, 0.9], [-0.2, 0.5, 0.1], [0.0, 0.0, 0.0]),
             ([tx0, 0.7], [ty0, -0.6], [0.5, 0.8]), (line, np.full(400, 0.37), np.full(400, 0.01)),
             (np.full(50, 3.5), np.full(50, -2.5), np.full(50, 0.02))]
    for xs, ys, ms in cases:
        lens = (0.1, 0.2, -0.05, np.array(xs, float), np.array(ys, float), np.array(ms, float))
        ox, oy, ob = ora.shoot(lens, rays, pix)
        s = ora.error_scale_block(lens, rays)
        with R.Context(lens) as ctx:
            ctx.set_expansion_block(block)
            ctx.set_expansion_cells(cells)
            gx, gy, gb = ctx.shoot(rays, "fp64_expansion", pix)
            gx, gy, gb = _np(gx), _np(gy), _np(gb)
            fin = np.isfinite(ox) & np.isfinite(oy)
            assert np.array_equal(fin, np.isfinite(gx) & np.isfinite(gy)), (xs, block)
            assert np.all(np.abs(gx[fin] - ox[fin]) <= BETA_TOL * s[fin])
            assert np.all(np.abs(gy[fin] - oy[fin]) <= BETA_TOL * s[fin])
            _assert_bins(gb, ob, _near_edges(ox, oy, s, pix))


@pytest.mark.parametrize("block", [1, 2, 4])
def test_expansion_star_cells_wide_field(torch, block):
    """20000 stars over a disk of radius 200 around a small lattice: most
    star cells lie far from every block and enter through their multipole
    expansions.  Per ray the result holds the FP64 bar against the oracle,
    with cells and without, and the two agree in every bin."""
    rng = np.random.default_rng(170)
    n = 20000
    r = 200.0 * np.sqrt(rng.random(n))
    phi = 2 * np.pi * rng.random(n)
    lens = (0.0, 0.1, 0.05, r * np.cos(phi), r * np.sin(phi), rng.uniform(0.05, 0.15, n))
    rays = (-3.0, -3.0, 6 / 256, 6 / 256, 256, 256, 0, 0)
    pix = (-2.5, -2.5, 5 / 64, 5 / 64, 64, 64)
    _say("oracle: 256^2 rays x 20000 stars")
    ox, oy, ob = ora.shoot(lens, rays, pix)
    s = ora.error_scale_block(lens, rays)
    bins = {}
    with R.Context(lens) as ctx:
        ctx.set_expansion_block(block)
        for cells in ("always", "never"):
            ctx.set_expansion_cells(cells)
            gx, gy, gb = ctx.shoot(rays, "fp64_expansion", pix)
            gx, gy, bins[cells] = _np(gx), _np(gy), _np(gb)
            assert np.all(np.abs(gx - ox) <= BETA_TOL * s), cells
            assert np.all(np.abs(gy - oy) <= BETA_TOL * s), cells
            _assert_bins(bins[cells], ob, _near_edges(ox, oy, s, pix), cells)
    assert np.array_equal(bins["always"], bins["never"])


def _oracle_threaded(lens, rays, pix, threads):
    """The oracle's per-ray results and error scale over a block of rays,
    split into row bands on host threads (ctypes releases the GIL around
    each call, and the oracle keeps no state between calls)."""
    from concurrent.futures import ThreadPoolExecutor
    ora.shoot(lens, rays.block(0, 0, 1, 1).as_tuple(), pix)   # loads the library once
    edges = [rays.ny * k // threads for k in range(threads + 1)]

    def run(k):
        sub = rays.block(0, edges[k], rays.nx, edges[k + 1] - edges[k]).as_tuple()
        bx, by, b = ora.shoot(lens, sub, pix)
        return bx, by, b, ora.error_scale_block(lens, sub)

    with ThreadPoolExecutor(threads) as pool:
        parts = list(pool.map(run, range(threads)))
    return [np.concatenate([p[i] for p in parts]) for i in range(4)]


def test_large_config_full_band_every_ray(torch):
    """A full-width band of the 8192^2 lattice of the large configuration
    (rows 3840..4351, 4.2e6 rays x 16384 stars): every ray against the
    oracle, for one-pass FP64, the expansion mode and FP32-bulk."""
    w = W.plain_fp64_large()
    band = w.rays.block(0, 3840, w.rays.nx, 512)
    threads = max(1, min(16, os.cpu_count() or 1))
    _say(f"oracle on {band.nx}x{band.ny} rays, {threads} threads")
    ox, oy, ob, s = _oracle_threaded(w.lens.as_tuple(), band, w.pix.as_tuple(), threads)
    near = _near_edges(ox, oy, s, w.pix.as_tuple())
    with R.Context(w.lens) as ctx:
        for prec in ("fp64", "fp64_expansion"):
            gx, gy, gb = (_np(t) for t in ctx.shoot(band, prec, w.pix))
            mis = np.count_nonzero(gb != ob)
            _say(prec, "misbinned", mis, "of", ob.size, "near edges", int(near.sum()), "max |dbeta|/S",
                 float(np.max(np.maximum(np.abs(gx - ox), np.abs(gy - oy)) / s)))
            assert np.all(np.abs(gx - ox) <= BETA_TOL * s), prec
            assert np.all(np.abs(gy - oy) <= BETA_TOL * s), prec
            _assert_bins(gb, ob, near, prec)
        _, _, fb = ctx.shoot(band, "fp32_bulk", w.pix, beta=False)
        frac = np.count_nonzero(_np(fb) != ob) / ob.size
        _say("fp32_bulk misbinned fraction against the oracle", frac)
        assert frac <= MISBIN_FP32


@pytest.mark.skipif(os.environ.get("RAYSH_FULL_LATTICE") != "1",
                    reason="about 4 minutes of oracle time on 16 host threads (the error scale takes a square "
                           "root and a division per interaction); run with RAYSH_FULL_LATTICE=1")
def test_large_config_whole_lattice_every_ray(torch):
    """Every ray of the 8192^2 lattice of the large configuration (6.7e7
    rays x 16384 stars, 1.1e12 interactions) against the oracle, band by
    band on the host's cores: one-pass FP64 and the expansion mode in the
    oracle's pixel (beta within 1e-12 S) away from pixel edges, FP32-bulk
    at most 1e-4 misbinned, and the FP64 map of the whole lattice (the
    launch the benchmark times) equal to the histogram of the oracle's bins
    up to the edge-band rays."""
    w = W.plain_fp64_large()
    pix = w.pix.as_tuple()
    threads = max(1, min(16, os.cpu_count() or 1))
    band_rows = 512
    want = np.zeros(w.pix.NX * w.pix.NY, np.int64)
    n_near = n32 = 0
    with R.Context(w.lens) as ctx:
        for j0 in range(0, w.rays.ny, band_rows):
            band = w.rays.block(0, j0, w.rays.nx, min(band_rows, w.rays.ny - j0))
            ox, oy, ob, sc = _oracle_threaded(w.lens.as_tuple(), band, pix, threads)
            near = _near_edges(ox, oy, sc, pix)
            n_near += int(near.sum())
            want += np.bincount(ob[ob >= 0].ravel(), minlength=want.size)
            worst = 0.0
            for prec in ("fp64", "fp64_expansion"):
                gx, gy, gb = (_np(t) for t in ctx.shoot(band, prec, w.pix))
                d = np.maximum(np.abs(gx - ox), np.abs(gy - oy)) / sc
                worst = max(worst, float(np.max(d)))
                assert np.all(d <= BETA_TOL), (prec, j0)
                _assert_bins(gb, ob, near, f"{prec} rows {j0}..")
            _, _, fb = ctx.shoot(band, "fp32_bulk", w.pix, beta=False)
            n32 += np.count_nonzero(_np(fb) != ob)
            _say(f"rows {j0}..{j0 + band.ny - 1}: max |dbeta|/S {worst:.2e}, near edges {int(near.sum())}")
        frac = n32 / (w.rays.nx * w.rays.ny)
        _say("fp32_bulk misbinned fraction against the oracle", frac)
        assert frac <= MISBIN_FP32
        m, nb = ctx.map(w.rays, w.pix, "fp64", n_binned=True)
        _assert_map(_np(m).ravel(), want, int(want.sum()), nb, n_near, "whole-lattice FP64 map")
