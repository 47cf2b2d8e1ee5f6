"""GPU parity of the surrogate's kernels against the FP64 oracle, and what the
trained network gains over the method without it."""
import math
import time

import numpy as np
import pytest

from oracle import surrogate as OS
from paper_1703_09707_amd import raysh as R
from paper_1703_09707_amd import surrogate as S
from paper_1703_09707_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return t


def _say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------- histogram
@pytest.fixture(scope="module")
def shot_map(torch):
    """A 256^2 map of the 100-star workload and its lattice."""
    w = W.plain_fp64_small()
    with R.Context(w.lens) as ctx:
        counts = ctx.map(w.rays, w.pix, "fp64")
    return w, counts


@pytest.mark.parametrize("sigma", [0.01, 0.05, 0.2, 1.0])
def test_histogram_matches_oracle(torch, shot_map, sigma):
    w, counts = shot_map
    norm = (w.rays.dx * w.rays.dy) / (w.pix.Px * w.pix.Py)
    mu_ref = W.mean_magnification(w.lens.kappa_c + w.lens.kappa_star, w.lens.gamma1, w.lens.gamma2)
    h = S.Histogrammer(w.pix.NX, w.pix.NY)
    bins, hist = h(counts, norm, sigma, w.pix.Px, w.pix.Py, mu_ref)
    got = bins.cpu().numpy().astype(np.int64)
    want_h, want_c, frac = OS.log_mag_histogram(counts.cpu().numpy(), w.rays.dx, w.rays.dy, w.pix.Px,
                                                w.pix.Py, sigma, mu_ref)
    near = int(np.count_nonzero(frac < 1e-9))
    assert got.sum() == want_c.sum()
    assert np.abs(got - want_c).sum() <= 2 * near, (near, np.abs(got - want_c).sum())
    np.testing.assert_allclose(hist.cpu().numpy(), got / got.sum(), rtol=1e-6, atol=1e-9)


def test_histogram_constant_map_and_errors(torch):
    c = torch.full((64, 64), 5, dtype=torch.int32, device="cuda")
    h = S.Histogrammer(64, 64)
    bins, hist = h(c, 0.2, 0.05, 0.1, 0.1, 1.0)   # mu = 1 everywhere -> log 0 -> bin 32
    b = bins.cpu().numpy()
    assert b[32] == b.sum() and b.sum() > 0
    assert hist.cpu().numpy()[32] == 1.0
    with pytest.raises(R.RayshError):
        h(c, 0.2, 5.0, 0.1, 0.1, 1.0)              # source larger than the map
    with pytest.raises(R.RayshError):
        h(c, 0.2, 0.05, 0.1, 0.1, 1.0, nbins=0)


# ----------------------------------------------------------------- network
def _net_case(seed=0, B=37, h=256):
    rng = np.random.default_rng(seed)
    params = OS.init_params(4, h, 64, rng)
    params = (params + rng.normal(0, 0.05, params.shape)).astype(np.float32)
    x = rng.standard_normal((B, 4)).astype(np.float32)
    t = rng.random((B, 64)).astype(np.float32)
    t /= t.sum(axis=1, keepdims=True)
    return params, x, t


def test_mlp_forward_matches_oracle(torch):
    params, x, _ = _net_case()
    net = S.MLP(params, max_batch=64)
    p = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    want, _ = OS.forward(params, x, 4, 256, 64)
    np.testing.assert_allclose(p, want, rtol=2e-4, atol=1e-7)
    net.close()


def test_mlp_gradient_matches_oracle(torch):
    params, x, t = _net_case(1)
    net = S.MLP(params, max_batch=64)
    g, loss = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    want = OS.gradients(params, x, t, 4, 256, 64)
    assert abs(loss.item() - OS.loss(params, x, t, 4, 256, 64)) < 1e-5
    err = np.linalg.norm(g - want) / np.linalg.norm(want)
    assert err < 1e-4, err
    np.testing.assert_allclose(g, want, rtol=1e-2, atol=1e-3 * np.abs(want).max())
    net.close()


def test_mlp_adam_matches_oracle(torch):
    params, x, t = _net_case(2)
    net = S.MLP(params, max_batch=64)
    xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    g1, _ = net.gradient(xg, tg)
    net.adam_step(1e-3)
    g2, _ = net.gradient(xg, tg)
    net.adam_step(1e-3)
    got = net.params()
    p, m, v = OS.adam(params, g1.cpu().numpy(), np.zeros_like(params), np.zeros_like(params), 1, 1e-3)
    p, m, v = OS.adam(p, g2.cpu().numpy(), m, v, 2, 1e-3)
    np.testing.assert_allclose(got, p, rtol=1e-6, atol=1e-7)
    # the forward pass uses the BF16 rounding of the updated masters
    want, _ = OS.forward(got, x, 4, 256, 64)
    np.testing.assert_allclose(net.forward(xg).cpu().numpy(), want, rtol=2e-4, atol=1e-7)
    net.close()


@pytest.mark.parametrize("n_in,h,n_out,B", [(3, 100, 37, 45), (7, 33, 65, 1), (1, 130, 5, 200), (9, 64, 17, 64)])
def test_mlp_ragged_sizes_match_oracle(torch, n_in, h, n_out, B):
    """Layer sizes and batches that are not multiples of the GEMM tiles
    (32 x 32 outputs, 64 deep) or of the column sums' 16 columns: forward,
    gradient and one Adam step against the oracle, at the full batch."""
    rng = np.random.default_rng(n_in * 1000 + h)
    params = OS.init_params(n_in, h, n_out, rng)
    params = (params + rng.normal(0, 0.05, params.shape)).astype(np.float32)
    x = rng.standard_normal((B, n_in)).astype(np.float32)
    t = rng.random((B, n_out)).astype(np.float32)
    t /= t.sum(axis=1, keepdims=True)
    net = S.MLP(params, n_in=n_in, n_hidden=h, n_out=n_out, max_batch=B)
    try:
        xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        want, _ = OS.forward(params, x, n_in, h, n_out)
        np.testing.assert_allclose(net.forward(xg).cpu().numpy(), want, rtol=2e-4, atol=1e-7)
        g, loss = net.gradient(xg, tg)
        g = g.cpu().numpy().astype(np.float64)
        gw = OS.gradients(params, x, t, n_in, h, n_out)
        assert abs(loss.item() - OS.loss(params, x, t, n_in, h, n_out)) < 1e-5
        assert np.linalg.norm(g - gw) / np.linalg.norm(gw) < 1e-4
        net.adam_step(1e-3)
        p, _, _ = OS.adam(params, g.astype(np.float32), np.zeros_like(params), np.zeros_like(params), 1, 1e-3)
        np.testing.assert_allclose(net.params(), p, rtol=1e-6, atol=1e-7)
    finally:
        net.close()


def test_mlp_rejects_bad_batch(torch):
    params, x, _ = _net_case()
    net = S.MLP(params, max_batch=16)
    with pytest.raises(R.RayshError):
        net.forward(torch.from_numpy(x).cuda())   # 37 rows > max_batch
    with pytest.raises(R.RayshError):
        net.adam_step(1e-3)                       # no gradient yet
    net.close()


# ----------------------------------------------------------------- learning
def test_network_beats_the_method_without_it(torch):
    """Small end-to-end run: shooter maps -> histograms -> training.  On
    held-out parameter sets the network's histograms are closer (L1) to the
    shooter's than the nearest training example's and than the training
    mean, and it answers orders of magnitude faster than shooting."""
    kw = dict(rays_per_side=2048, npix=256, sigmas_per_map=4, n_lo=200, n_hi=6000)
    t0 = time.perf_counter()
    train = S.generate(384, seed=11, **kw)
    test = S.generate(48, seed=12, **kw)
    _say(f"data: {len(train.hist)} train, {len(test.hist)} test examples, {time.perf_counter() - t0:.1f} s")
    net, std, hist = S.train(train, steps=2500, batch=256, lr=2e-3)
    res, _ = S.evaluate(net, std, train, test)
    x = torch.from_numpy(std(test.features)).cuda()
    assert x.shape[0] <= net.max_batch
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(10):
        net.forward(x)
    torch.cuda.synchronize()
    per_example = (time.perf_counter() - t1) / (10 * len(test.hist))
    shoot_per_map = test.seconds_shooting / (len(test.hist) / 4)
    _say("loss", hist[0], hist[-1], res, f"predict {per_example * 1e6:.2f} us/example",
         f"shoot {shoot_per_map * 1e3:.2f} ms/map")
    assert hist[-1][1] < hist[0][1]
    assert res["l1_network"] < res["l1_training_mean"]
    assert res["l1_network"] < res["l1_nearest_neighbour"]
    assert per_example * 100 < shoot_per_map
    net.close()


def test_generate_with_expansion_maps_matches_direct(torch):
    """Training data shot with the far-field expansion is the data the
    direct FP64 sum gives (the two bin the same rays up to the FP64 bar)."""
    kw = dict(rays_per_side=1024, npix=256, sigmas_per_map=2, n_lo=300, n_hi=3000)
    direct = S.generate(6, seed=31, precision="fp64", **kw)
    fast = S.generate(6, seed=31, precision="fp64_expansion", **kw)
    assert np.array_equal(direct.features, fast.features)
    l1 = np.abs(direct.hist - fast.hist).sum(axis=1)
    _say("expansion vs direct histograms: max L1", float(l1.max()),
         f"shooting {direct.seconds_shooting:.3f} s direct, {fast.seconds_shooting:.3f} s expansion")
    assert l1.max() < 1e-4


# ----------------------------------------------------------------- the surrogate and its fallback
def test_surrogate_falls_back_to_the_shooter_outside_its_domain(torch):
    """Queries inside the training domain are answered by the network,
    queries outside it by the plain shooter (the fallback), bit for bit what
    shooting them gives; a query the shooter cannot answer either raises."""
    kw = dict(rays_per_side=512, npix=128, sigmas_per_map=2, n_lo=200, n_hi=3000)
    train = S.generate(48, seed=21, **kw)
    net, std, _ = S.train(train, steps=200, batch=64, lr=2e-3)
    cfg = S.ShooterConfig(rays_per_side=512, npix=128, precision="fp64")
    sur = S.Surrogate(net, std, train, cfg, seed=77)
    inside = train.features[:5].astype(np.float64)            # training examples: in the domain
    outside = np.array([[0.9, 0.05, 0.5, -1.0],                # kappa above the training box
                        [0.5, 0.3, 0.6, 0.05]])                # sigma above it
    h, src = sur.query(np.concatenate([inside, outside]))
    assert src.tolist() == ["network"] * 5 + ["shooter"] * 2
    np.testing.assert_array_equal(h[:5], S.predict(net, std, inside))
    want = S.shoot_histograms(outside, cfg, seed=77)
    np.testing.assert_array_equal(h[5:], want)
    assert np.allclose(h.sum(axis=1), 1.0, atol=1e-5)
    # the fallback's histogram is the plain shooter's: the same map shot by hand
    rng = np.random.Generator(np.random.PCG64(77))
    lens, hx, hy = S.lens_for(0.9, 0.05, 0.5, cfg.window, rng)
    grid = W.centred_rays(hx, hy, cfg.rays_per_side, cfg.rays_per_side)
    pix = W.centred_window(cfg.window, cfg.npix)
    with R.Context(lens) as ctx:
        counts = ctx.map(grid, pix, "fp64")
    _, h0 = S.Histogrammer(cfg.npix, cfg.npix)(counts, (grid.dx * grid.dy) / (pix.Px * pix.Py), 0.1, pix.Px,
                                                pix.Py, W.mean_magnification(0.9, 0.05, 0.0))
    np.testing.assert_array_equal(h[5], h0.cpu().numpy())
    with pytest.raises(ValueError):
        sur.query([[1.2, 0.2, 0.5, -1.0]])                     # outside the domain and critical: det A = 0
    with pytest.raises(ValueError):
        sur.query([[0.5, 0.3, 0.6, 0.6]])                      # a source too wide for the window
    net.close()
