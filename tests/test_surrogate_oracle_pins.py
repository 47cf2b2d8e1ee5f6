"""Pins of the surrogate's FP64 oracle (map -> histogram, network, Adam)."""
import math

import numpy as np
import pytest

from oracle import shooter as ora
from oracle import surrogate as S_REAL


# ----------------------------------------------------------------- map -> histogram
def pin_magnification_of_a_sheet_is_inverse_determinant(S):
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


def pin_gaussian_taps(S):
    for sigma, pixel in ((0.01, 0.0195), (0.1, 0.0195), (1.0, 0.0195), (0.3, 0.05)):
        g, r = S.gaussian_taps(sigma, pixel)
        assert len(g) == 2 * r + 1 and r == math.ceil(3 * sigma / pixel)
        assert abs(g.sum() - 1) < 1e-14
        np.testing.assert_array_equal(g, g[::-1])
        if sigma > 5 * pixel:   # the sampled variance is sigma^2 up to the truncation near 3 sigma
            k = np.arange(-r, r + 1) * pixel
            assert abs((g * k * k).sum() / sigma ** 2 - 1) < 0.04


def pin_smooth_constant_delta_and_ramp(S):
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


def pin_histogram_bins_of_known_values(S):
    nb, lo, hi = 64, -2.0, 2.0
    mu_ref = 2.5
    vals = np.array([[0.0, mu_ref, 10 * mu_ref, 1e-3 * mu_ref, 1e3 * mu_ref, 0.999 * mu_ref]])
    b, frac = S.log_mag_bins(vals, mu_ref, nb, lo, hi)
    assert b.tolist() == [[0, 32, 48, 0, 63, 31]]
    assert frac[0, 1] == 0.0 and frac[0, 2] < 1e-12   # exactly on edges
    h, hc, _ = S.log_mag_histogram(np.full((30, 30), 7), 0.1, 0.1, 0.1, 0.1, 0.05, 7.0)
    assert hc.sum() > 0 and h[32] == 1.0 and abs(h.sum() - 1) < 1e-15


# ----------------------------------------------------------------- network
def pin_bf16_rounding_matches_torch(S):
    import torch
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-5, 5, 20000)).astype(np.float32)
    ties = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0 + 2 ** -7], np.float32)
    a = np.concatenate([a, ties])
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16_round(a), want)
    assert S.bf16_round(ties).tolist() == [1.0, 1.0 + 2 ** -6, -1.0, 3.0]


def pin_gelu_matches_torch_and_its_derivative(S):
    import torch
    z = np.linspace(-6, 6, 1001)
    want = torch.nn.functional.gelu(torch.from_numpy(z)).numpy()
    np.testing.assert_allclose(S.gelu(z), want, rtol=1e-12, atol=1e-15)
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    assert S.gelu(0.0) == 0.0 and S.gelu_grad(0.0) == 0.5


def _tiny(S, seed=0, n_in=4, h=8, n_out=5, B=6):
    rng = np.random.default_rng(seed)
    params = S.init_params(n_in, h, n_out, rng).astype(np.float64)
    params += rng.normal(0, 0.1, params.shape)   # non-zero biases too
    x = rng.standard_normal((B, n_in))
    t = rng.random((B, n_out))
    t /= t.sum(axis=1, keepdims=True)
    return params, x, t, (n_in, h, n_out)


def pin_gradients_match_finite_differences(S):
    params, x, t, dims = _tiny(S)
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


def pin_softmax_cross_entropy_special_cases(S):
    params, x, _, dims = _tiny(S, 1)
    p, _ = S.forward(params, x, *dims, weights_bf16=False)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=1e-15)
    # target = prediction: the loss is the mean entropy and the gradient vanishes
    ent = -(p * np.log(p)).sum(axis=1).mean()
    assert abs(S.loss(params, x, p, *dims, weights_bf16=False) - ent) < 1e-13
    assert np.abs(S.gradients(params, x, p, *dims, weights_bf16=False)).max() < 1e-15
    onehot = np.eye(dims[2])[np.arange(len(x)) % dims[2]]
    want = -np.log(p[np.arange(len(x)), np.arange(len(x)) % dims[2]]).mean()
    assert abs(S.loss(params, x, onehot, *dims, weights_bf16=False) - want) < 1e-13


def pin_adam_first_step_is_signed_learning_rate(S):
    g = np.array([3.0, -0.2, 1e-3, -7.0])
    p, m, v = S.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def pin_adam_constant_gradient(S):
    """A constant gradient g from the zero state: the moments are the
    geometric sums m_t = (1 - beta1^t) g and v_t = (1 - beta2^t) g^2, so the
    bias-corrected moments are exactly g and g^2 at every step and, with
    eps = 0, every step moves each parameter by lr against the sign of its
    gradient.  A beta1 and beta2 swapped anywhere in the recurrences or the
    corrections breaks this from the second step on."""
    g = np.array([3.0, -0.2, 1e-3, -7.0])
    lr, b1, b2 = 0.01, 0.9, 0.999
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 7):
        p, m, v = S.adam(p, g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=0.0)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(p, -lr * t * np.sign(g), rtol=1e-12)


def pin_adam_three_steps_from_a_nonzero_state(S):
    """Three steps with different gradients from a state (m0, v0) reached at
    step 4: the moments equal their unrolled exponential averages
    beta^n x0 + (1 - beta) sum_u beta^(n-u) g_u (a sum over the gradient
    history, not the one-step recurrence), and each parameter update is
    lr * mhat / (sqrt(vhat) + eps) with the bias corrections of steps 5, 6
    and 7."""
    rng = np.random.default_rng(12)
    n = 7
    p0 = rng.normal(0, 1, n)
    m0 = rng.normal(0, 0.3, n)
    v0 = rng.uniform(0.1, 2.0, n)
    gs = [rng.normal(0, 1, n) for _ in range(3)]
    lr, b1, b2, eps = 3e-3, 0.8, 0.95, 1e-6
    p, m, v = p0, m0, v0
    want_p = p0.copy()
    for k in range(1, 4):
        p, m, v = S.adam(p, gs[k - 1], m, v, 4 + k, lr=lr, beta1=b1, beta2=b2, eps=eps)
        mk = b1 ** k * m0 + (1 - b1) * sum(b1 ** (k - u) * gs[u - 1] for u in range(1, k + 1))
        vk = b2 ** k * v0 + (1 - b2) * sum(b2 ** (k - u) * gs[u - 1] ** 2 for u in range(1, k + 1))
        np.testing.assert_allclose(m, mk, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(v, vk, rtol=1e-12)
        want_p = want_p - lr * (mk / (1 - b1 ** (4 + k))) / (np.sqrt(vk / (1 - b2 ** (4 + k))) + eps)
        np.testing.assert_allclose(p, want_p, rtol=1e-12, atol=1e-15)


PINS = [pin_magnification_of_a_sheet_is_inverse_determinant, pin_gaussian_taps, pin_smooth_constant_delta_and_ramp,
        pin_histogram_bins_of_known_values, pin_bf16_rounding_matches_torch,
        pin_gelu_matches_torch_and_its_derivative, pin_gradients_match_finite_differences,
        pin_softmax_cross_entropy_special_cases, pin_adam_first_step_is_signed_learning_rate,
        pin_adam_constant_gradient, pin_adam_three_steps_from_a_nonzero_state]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(S_REAL)
