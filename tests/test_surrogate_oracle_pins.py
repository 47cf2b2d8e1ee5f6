"""Pins of the surrogate's FP64 oracle (map -> histogram, network, Adam)."""
import math

import numpy as np
import pytest

from oracle import shooter as ora
from oracle import surrogate as S


# ----------------------------------------------------------------- map -> histogram
def test_magnification_of_a_sheet_is_inverse_determinant(oracle_lib):
    """No stars: the normalised counts equal 1/|det A| in every pixel far
    from the window edge (to lattice-counting error)."""
    kc, g1, g2 = 0.25, 0.125, 0.0
    det = (1 - kc) ** 2 - g1 ** 2
    rays = (-4.0, -4.0, 8 / 1600, 8 / 1600, 1600, 1600, 0, 0)
    pix = (-1.0, -1.0, 0.125, 0.125, 16, 16)
    counts, _ = ora.map_counts((kc, g1, g2, [], [], []), rays, pix)
    mu = S.magnification(counts, rays[2], rays[3], pix[2], pix[3])
    np.testing.assert_allclose(mu, 1.0 / det, rtol=0.02)
    assert abs(mu.mean() * det - 1) < 2e-3


@pytest.mark.parametrize("sigma,pixel", [(0.01, 0.0195), (0.1, 0.0195), (1.0, 0.0195), (0.3, 0.05)])
def test_gaussian_taps(sigma, pixel):
    g, r = S.gaussian_taps(sigma, pixel)
    assert len(g) == 2 * r + 1 and r == math.ceil(3 * sigma / pixel)
    assert abs(g.sum() - 1) < 1e-14
    np.testing.assert_array_equal(g, g[::-1])
    if sigma > 5 * pixel:   # the sampled variance is sigma^2 up to the truncation near 3 sigma
        k = np.arange(-r, r + 1) * pixel
        assert abs((g * k * k).sum() / sigma ** 2 - 1) < 0.04


def test_smooth_constant_delta_and_ramp():
    ny, nx, P, sigma = 40, 50, 0.1, 0.25
    out = S.smooth(np.full((ny, nx), 3.0), sigma, P, P)
    np.testing.assert_allclose(out, 3.0, rtol=1e-14)
    g, r = S.gaussian_taps(sigma, P)
    d = np.zeros((ny, nx))
    d[20, 25] = 1.0
    out = S.smooth(d, sigma, P, P)
    want = np.zeros_like(out)
    want[20 - 2 * r:20 + 1, 25 - 2 * r:25 + 1] = np.outer(g[::-1], g[::-1])
    np.testing.assert_allclose(out, want, atol=1e-16)
    assert abs(out.sum() - 1) < 1e-14
    ramp = np.tile(np.arange(nx, dtype=np.float64), (ny, 1))
    out = S.smooth(ramp, sigma, P, P)
    np.testing.assert_allclose(out, ramp[r:ny - r, r:nx - r], rtol=1e-13)


def test_histogram_bins_of_known_values():
    nb, lo, hi = 64, -2.0, 2.0
    mu_ref = 2.5
    vals = np.array([[0.0, mu_ref, 10 * mu_ref, 1e-3 * mu_ref, 1e3 * mu_ref, 0.999 * mu_ref]])
    b, frac = S.log_mag_bins(vals, mu_ref, nb, lo, hi)
    assert b.tolist() == [[0, 32, 48, 0, 63, 31]]
    assert frac[0, 1] == 0.0 and frac[0, 2] < 1e-12   # exactly on edges
    h, hc, _ = S.log_mag_histogram(np.full((30, 30), 7), 0.1, 0.1, 0.1, 0.1, 0.05, 7.0)
    assert hc.sum() > 0 and h[32] == 1.0 and abs(h.sum() - 1) < 1e-15


# ----------------------------------------------------------------- network
def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-5, 5, 20000)).astype(np.float32)
    ties = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0 + 2 ** -7], np.float32)
    a = np.concatenate([a, ties])
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16_round(a), want)
    assert S.bf16_round(ties).tolist() == [1.0, 1.0 + 2 ** -6, -1.0, 3.0]


def test_gelu_matches_torch_and_its_derivative():
    import torch
    z = np.linspace(-6, 6, 1001)
    want = torch.nn.functional.gelu(torch.from_numpy(z)).numpy()
    np.testing.assert_allclose(S.gelu(z), want, rtol=1e-12, atol=1e-15)
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    assert S.gelu(0.0) == 0.0 and S.gelu_grad(0.0) == 0.5


def _tiny(seed=0, n_in=4, h=8, n_out=5, B=6):
    rng = np.random.default_rng(seed)
    params = S.init_params(n_in, h, n_out, rng).astype(np.float64)
    params += rng.normal(0, 0.1, params.shape)   # non-zero biases too
    x = rng.standard_normal((B, n_in))
    t = rng.random((B, n_out))
    t /= t.sum(axis=1, keepdims=True)
    return params, x, t, (n_in, h, n_out)


def test_gradients_match_finite_differences():
    params, x, t, dims = _tiny()
    g = S.gradients(params, x, t, *dims, weights_bf16=False)
    eps = 1e-6
    fd = np.empty_like(params)
    for i in range(len(params)):
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        fd[i] = (S.loss(p1, x, t, *dims, weights_bf16=False) -
                 S.loss(p2, x, t, *dims, weights_bf16=False)) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_softmax_cross_entropy_special_cases():
    params, x, _, dims = _tiny(1)
    p, _ = S.forward(params, x, *dims, weights_bf16=False)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=1e-15)
    # target = prediction: the loss is the mean entropy and the gradient vanishes
    ent = -(p * np.log(p)).sum(axis=1).mean()
    assert abs(S.loss(params, x, p, *dims, weights_bf16=False) - ent) < 1e-13
    assert np.abs(S.gradients(params, x, p, *dims, weights_bf16=False)).max() < 1e-15
    onehot = np.eye(dims[2])[np.arange(len(x)) % dims[2]]
    want = -np.log(p[np.arange(len(x)), np.arange(len(x)) % dims[2]]).mean()
    assert abs(S.loss(params, x, onehot, *dims, weights_bf16=False) - want) < 1e-13


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.2, 1e-3, -7.0])
    p, m, v = S.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
