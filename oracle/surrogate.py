"""FP64 oracle of the surrogate's data and network steps: TEST INFRASTRUCTURE ONLY.

Maps from backward ray shooting are turned into magnification histograms,
and a small network learns them for the parameter-space exploration of the
Bayesian Monte Carlo analysis (arXiv:1703.09707, Sec. 1).

Map -> histogram:
  * The ray count of a pixel is proportional to the magnification of a
    source there (Sec. 1).  Without lensing a pixel receives
    Px*Py / (dx*dy) rays, so mu = counts * (dx*dy) / (Px*Py).
  * A source of finite size sees the map convolved with its profile
    (Sec. 1).  The profile here is a circular Gaussian of width sigma,
    sampled at pixel offsets k*P for |k| <= r = ceil(3 sigma / P) and
    normalised to unit sum on each axis (separable).  Only pixels at least
    r from every edge are kept.
  * The histogram has `nbins` uniform bins of log10(mu_sigma / mu_ref) on
    [lo, hi).  Values below lo (mu_sigma = 0 included) go to the first
    bin and values at or above hi to the last.  The histogram is normalised
    to unit sum.

Network: layers n_in -> h -> h -> n_out with GELU (exact, erf form) after
the first two, softmax output, cross-entropy against a target histogram
averaged over the batch, and Adam with FP32 master weights whose BF16
rounding (round to nearest, ties to even) is what the forward pass uses.
Weights are stored W[in][out], row-major.
"""
import math

import numpy as np
from scipy import special


# ----------------------------------------------------------------- map -> histogram
def magnification(counts, dx, dy, px, py):
    return np.asarray(counts, np.float64) * ((dx * dy) / (px * py))


def gaussian_taps(sigma, pixel):
    """Normalised 1D taps g[0..2r] at offsets (k - r) * pixel, and r."""
    r = int(math.ceil(3.0 * sigma / pixel))
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-0.5 * ((k * pixel) / sigma) ** 2)
    return g / g.sum(), r


def smooth(mu, sigma, px, py):
    """Separable Gaussian convolution, rows first, taps in increasing k;
    returns the valid interior (ny - 2ry, nx - 2rx)."""
    gx, rx = gaussian_taps(sigma, px)
    gy, ry = gaussian_taps(sigma, py)
    ny, nx = mu.shape
    wx, wy = nx - 2 * rx, ny - 2 * ry
    if wx <= 0 or wy <= 0:
        raise ValueError("source larger than the map")
    tmp = np.zeros((ny, wx), np.float64)
    for k in range(2 * rx + 1):
        tmp += gx[k] * mu[:, k:k + wx]
    out = np.zeros((wy, wx), np.float64)
    for k in range(2 * ry + 1):
        out += gy[k] * tmp[k:k + wy, :]
    return out


def log_mag_bins(mu_s, mu_ref, nbins=64, lo=-2.0, hi=2.0):
    """Bin index of every pixel and the distance of its coordinate to the
    nearest bin edge (in bins)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = np.where(mu_s > 0, np.log10(np.where(mu_s > 0, mu_s, 1.0) / mu_ref), -np.inf)
        u = (v - lo) / (hi - lo) * nbins
        b = np.floor(np.where(np.isfinite(u), u, -1.0))
        b = np.clip(b, 0, nbins - 1).astype(np.int64)
        frac = np.where(np.isfinite(u), np.abs(u - np.round(u)), np.inf)
    return b, frac


def log_mag_histogram(counts, dx, dy, px, py, sigma, mu_ref, nbins=64, lo=-2.0, hi=2.0):
    """(normalised histogram, integer counts per bin, edge distance per pixel)."""
    mu = magnification(counts, dx, dy, px, py)
    mu_s = smooth(mu, sigma, px, py)
    b, frac = log_mag_bins(mu_s, mu_ref, nbins, lo, hi)
    h = np.bincount(b.ravel(), minlength=nbins)
    return h / h.sum(), h, frac


# ----------------------------------------------------------------- network
def bf16_round(a):
    """Round FP32 values to BF16 (nearest, ties to even); returned as FP64."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def layer_shapes(n_in, h, n_out):
    return [(n_in, h), (h,), (h, h), (h,), (h, n_out), (n_out,)]


def unflatten(flat, n_in, h, n_out):
    out, o = [], 0
    for s in layer_shapes(n_in, h, n_out):
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], np.float64).reshape(s))
        o += n
    return out


def n_params(n_in, h, n_out):
    return sum(int(np.prod(s)) for s in layer_shapes(n_in, h, n_out))


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, x, n_in, h, n_out, weights_bf16=True):
    """Softmax probabilities and the intermediates of the backward pass.
    params: flat FP32 masters; weights are used BF16-rounded, biases as they are."""
    W1, b1, W2, b2, W3, b3 = unflatten(params, n_in, h, n_out)
    if weights_bf16:
        W1, W2, W3 = bf16_round(W1), bf16_round(W2), bf16_round(W3)
    x = np.asarray(x, np.float64)
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    z3 = h2 @ W3 + b3
    z3m = z3 - z3.max(axis=1, keepdims=True)
    e = np.exp(z3m)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (x, z1, h1, z2, h2, z3, W1, W2, W3)


def loss(params, x, t, n_in, h, n_out, weights_bf16=True):
    """Cross-entropy -mean_b sum_j t_bj log p_bj."""
    p, (_, _, _, _, _, z3, _, _, _) = forward(params, x, n_in, h, n_out, weights_bf16)
    z3m = z3 - z3.max(axis=1, keepdims=True)
    logp = z3m - np.log(np.exp(z3m).sum(axis=1, keepdims=True))
    return float(-(np.asarray(t, np.float64) * logp).sum() / len(x))


def gradients(params, x, t, n_in, h, n_out, weights_bf16=True):
    """Gradient of `loss` with respect to the flat parameters (the BF16
    rounding of the weights is treated as the identity, as in training)."""
    p, (x, z1, h1, z2, h2, z3, W1, W2, W3) = forward(params, x, n_in, h, n_out, weights_bf16)
    B = len(x)
    dz3 = (p - np.asarray(t, np.float64)) / B
    dW3 = h2.T @ dz3
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ W3.T) * gelu_grad(z2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new (params, m, v)."""
    g = np.asarray(grads, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return np.asarray(params, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(n_in, h, n_out, rng):
    """Deterministic He-style initialisation (FP32 masters)."""
    out = []
    for s in layer_shapes(n_in, h, n_out):
        if len(s) == 2:
            out.append(rng.normal(0.0, math.sqrt(2.0 / s[0]), s))
        else:
            out.append(np.zeros(s))
    return np.concatenate([a.ravel() for a in out]).astype(np.float32)
