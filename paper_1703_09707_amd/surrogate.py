"""Learned surrogate for magnification histograms (binding and host driver).

The Bayesian Monte Carlo analysis that motivates fast map generation
(arXiv:1703.09707, Sec. 1) needs the magnification statistics of many lens
parameter sets.  Here the shooter generates maps over sampled
(kappa, gamma, kappa_*/kappa); each map, seen by Gaussian sources of several
sizes, gives a 64-bin histogram of log10(mu_sigma / mu_macro); a small network
(4 -> 256 -> 256 -> 64, BF16 weights, FP32 accumulation) learns to predict
the histogram from (kappa, gamma, kappa_*/kappa, log10 sigma).  The shooter
remains the judge: held-out histograms are compared by L1 distance with the
network's predictions, with the realisation-noise floor (two star fields at
the same parameters) and with a no-network baseline (the nearest training
example in standardised feature space).

Every numerical step runs in libraysh's kernels (raysh_map_batch, or
raysh_map per set for the expansion mode, raysh_log_mag_histogram,
raysh_mlp_*); this module marshals arguments, draws parameters and loops
over batches.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import time

import numpy as np

from . import raysh as R
from . import workloads as W

N_FEATURES = 4
N_BINS = 64
LOG_RANGE = (-2.0, 2.0)
SIGMA_RANGE = (0.01, 1.0)


def _torch():
    return R._torch()


# ----------------------------------------------------------------- histogram
class Histogrammer:
    """raysh_log_mag_histogram with a reusable device workspace."""

    def __init__(self, nx, ny, device=0):
        torch = _torch()
        lib = R.load()
        self.nx, self.ny = int(nx), int(ny)
        nbytes = lib.raysh_histogram_workspace(self.nx, self.ny)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=torch.device("cuda", device))
        self.device = device

    def __call__(self, counts, norm, sigma, px, py, mu_ref, nbins=N_BINS, lo=LOG_RANGE[0],
                 hi=LOG_RANGE[1], stream=None, out=None):
        """Returns (bin counts int32[nbins], normalised float32[nbins]) device tensors."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        if out is None:
            out = (torch.empty(nbins, dtype=torch.int32, device=dev),
                   torch.empty(nbins, dtype=torch.float32, device=dev))
        bins, hist = out
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        R.check(R.load().raysh_log_mag_histogram(
            ctypes.c_void_p(counts.data_ptr()), self.nx, self.ny, float(norm), float(sigma), float(px),
            float(py), float(mu_ref), int(nbins), float(lo), float(hi),
            ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
            ctypes.c_void_p(bins.data_ptr()), ctypes.c_void_p(hist.data_ptr()) if hist is not None else None,
            ctypes.c_void_p(s.cuda_stream)))
        return bins, hist


# ----------------------------------------------------------------- network
class MLP:
    """raysh_mlp: n_in -> h -> h -> n_out, GELU, softmax; BF16 weights."""

    def __init__(self, params, n_in=N_FEATURES, n_hidden=256, n_out=N_BINS, max_batch=1024, device=0,
                 stream=None):
        torch = _torch()
        lib = R.load()
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.dims = (int(n_in), int(n_hidden), int(n_out))
        self.device = device
        self.max_batch = int(max_batch)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._ptr = ctypes.c_void_p()
        R.check(lib.raysh_mlp_create(ctypes.byref(self._ptr), device, ctypes.c_void_p(s.cuda_stream),
                                     *self.dims, self.max_batch, p.ctypes.data))
        self.n_params = int(lib.raysh_mlp_n_params(self._ptr))
        assert self.n_params == len(p)
        dev = torch.device("cuda", device)
        self._loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def forward(self, x, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((x.shape[0], self.dims[2]), dtype=torch.float32, device=x.device)
        R.check(R.load().raysh_mlp_forward(self._ptr, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                           ctypes.c_void_p(out.data_ptr())))
        return out

    def gradient(self, x, t):
        """(gradient float32[n_params], loss float32[1]) device tensors."""
        torch = _torch()
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        R.check(R.load().raysh_mlp_gradient(self._ptr, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(t.data_ptr()), int(x.shape[0]),
                                            ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr())))
        return g, loss

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        R.check(R.load().raysh_mlp_adam_step(self._ptr, lr, beta1, beta2, eps))

    def train_step(self, x, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One gradient + Adam step; returns the device loss tensor (the
        batch's loss before the step)."""
        R.check(R.load().raysh_mlp_train_step(self._ptr, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(t.data_ptr()), int(x.shape[0]), lr, beta1,
                                              beta2, eps, ctypes.c_void_p(self._loss.data_ptr())))
        return self._loss

    def params(self):
        out = np.empty(self.n_params, np.float32)
        R.check(R.load().raysh_mlp_get_params(self._ptr, out.ctypes.data))
        return out

    def close(self):
        if self._ptr:
            R.check(R.load().raysh_mlp_free(self._ptr))
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._ptr:
                R.load().raysh_mlp_free(self._ptr)
        except Exception:
            pass


def init_params(n_in=N_FEATURES, h=256, n_out=N_BINS, seed=0):
    """He-normal weights, zero biases, flat in the library's layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in [(n_in, h), (h,), (h, h), (h,), (h, n_out), (n_out,)]:
        if len(shape) == 2:
            parts.append(rng.normal(0.0, math.sqrt(2.0 / shape[0]), shape))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


# ----------------------------------------------------------------- data
@dataclasses.dataclass
class Dataset:
    features: np.ndarray      # [N, 4]: kappa, gamma, kappa_star/kappa, log10 sigma
    hist: np.ndarray          # [N, 64] normalised
    set_index: np.ndarray     # [N] parameter set of each example
    seconds_shooting: float
    seconds_histogram: float
    interactions: int
    rays: int


def sample_sigmas(rng, n):
    lo, hi = (math.log(v) for v in SIGMA_RANGE)
    return np.exp(rng.uniform(lo, hi, n))


def generate(n_sets, seed, rays_per_side=4096, npix=512, window=10.0, sigmas_per_map=4,
             precision="fp32_bulk", chunk=64, device=0, star_seed_offset=0, params=None,
             n_lo=500, n_hi=50000, log=None):
    """Shoot n_sets maps (lens parameters drawn as in workloads.draw_batch_params)
    and histogram each under sigmas_per_map Gaussian sources.  With `params`
    (a list of parameter dicts) the given sets are shot instead, with star
    fields seeded by seed + star_seed_offset.  The maps of a chunk are shot in
    one batched launch ("fp64", "fp32_bulk") or one expansion-mode launch per
    set ("fp64_expansion")."""
    torch = _torch()
    rng = np.random.Generator(np.random.PCG64(seed))
    if params is None:
        params, _ = W.draw_batch_params(rng, n_sets, n_lo, n_hi, window)
    sig_rng = np.random.Generator(np.random.PCG64(seed + 7))
    pix = W.centred_window(window, npix)
    hist = Histogrammer(npix, npix, device)
    feats, hists, sets = [], [], []
    t_shoot = t_hist = 0.0
    inter = rays = 0
    for c0 in range(0, len(params), chunk):
        part = params[c0:c0 + chunk]
        ctxs, grids = [], []
        for s, p in enumerate(part):
            srng = np.random.Generator(np.random.PCG64(seed + star_seed_offset + 1000 + c0 + s))
            m = W.salpeter_masses(p["n_stars"], srng)
            x, y, _ = W.star_field(m, p["kappa_star"], srng)
            ctxs.append(R.Context((p["kappa_c"], p["gamma"], 0.0, x, y, m), device=device))
            grids.append(W.centred_rays(p["hx"], p["hy"], rays_per_side, rays_per_side))
            inter += rays_per_side ** 2 * p["n_stars"]
            rays += rays_per_side ** 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if precision == "fp64_expansion":
            maps = [c.map(g, pix, precision) for c, g in zip(ctxs, grids)]
        else:
            maps = R.map_batch(ctxs, grids, [pix] * len(part), precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_shoot += t1 - t0
        sig = sample_sigmas(sig_rng, len(part) * sigmas_per_map).reshape(len(part), sigmas_per_map)
        out = torch.empty((len(part) * sigmas_per_map, N_BINS), dtype=torch.float32, device="cuda")
        bins = torch.empty(N_BINS, dtype=torch.int32, device="cuda")
        for s, p in enumerate(part):
            g = grids[s]
            norm = (g.dx * g.dy) / (pix.Px * pix.Py)
            mu_ref = W.mean_magnification(p["kappa"], p["gamma"], 0.0)
            for q in range(sigmas_per_map):
                hist(maps[s], norm, sig[s, q], pix.Px, pix.Py, mu_ref,
                     out=(bins, out[s * sigmas_per_map + q]))
                feats.append([p["kappa"], p["gamma"], p["f"], math.log10(sig[s, q])])
                sets.append(c0 + s)
        hists.append(out.cpu().numpy())
        torch.cuda.synchronize()
        t_hist += time.perf_counter() - t1
        for c in ctxs:
            c.close()
        if log:
            log(f"  shot sets {c0}..{c0 + len(part) - 1} ({t_shoot:.1f} s shooting)")
    return Dataset(np.asarray(feats, np.float32), np.concatenate(hists), np.asarray(sets), t_shoot, t_hist,
                   inter, rays)


@dataclasses.dataclass
class Standardiser:
    mean: np.ndarray
    std: np.ndarray

    @classmethod
    def fit(cls, x):
        return cls(x.mean(axis=0), x.std(axis=0) + 1e-12)

    def __call__(self, x):
        return ((x - self.mean) / self.std).astype(np.float32)


def l1(p, q):
    """L1 distance of histograms, row by row (in [0, 2])."""
    return np.abs(np.asarray(p, np.float64) - np.asarray(q, np.float64)).sum(axis=-1)


def nearest_neighbour(train_x, train_y, query_x):
    """No-network baseline: the histogram of the nearest training example."""
    d = ((query_x[:, None, :] - train_x[None, :, :]) ** 2).sum(-1)
    return train_y[d.argmin(axis=1)]


def train(data: Dataset, steps=3000, batch=256, lr=2e-3, hidden=256, seed=0, device=0, log=None):
    """Train the network on the dataset with the library's kernels; returns
    (MLP, Standardiser, loss history)."""
    torch = _torch()
    std = Standardiser.fit(data.features)
    X = torch.from_numpy(std(data.features)).to(f"cuda:{device}")
    Y = torch.from_numpy(data.hist.astype(np.float32)).to(f"cuda:{device}")
    net = MLP(init_params(N_FEATURES, hidden, N_BINS, seed), n_hidden=hidden, max_batch=batch, device=device)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    hist = []
    for step in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(X.device)
        xb, yb = X[idx].contiguous(), Y[idx].contiguous()
        rate = lr * 0.5 * (1 + math.cos(math.pi * step / steps))   # cosine decay
        loss = net.train_step(xb, yb, rate)
        if step % 200 == 0 or step == steps - 1:
            hist.append((step, float(loss.item())))
            if log:
                log(f"  step {step} loss {hist[-1][1]:.4f}")
    return net, std, hist


def predict(net: MLP, std: Standardiser, features):
    torch = _torch()
    x = torch.from_numpy(std(np.asarray(features, np.float32))).to(f"cuda:{net.device}")
    out = []
    for i in range(0, x.shape[0], net.max_batch):
        out.append(net.forward(x[i:i + net.max_batch].contiguous()))
    return torch.cat(out).cpu().numpy()


def evaluate(net, std, train_data: Dataset, test_data: Dataset, noise_data: Dataset | None = None):
    """Held-out L1 of the network, of the nearest-neighbour baseline and of
    the training-mean histogram; with noise_data (the test sets shot again
    with other star fields, same sources) also the realisation-noise floor."""
    pred = predict(net, std, test_data.features)
    nn = nearest_neighbour(std(train_data.features), train_data.hist, std(test_data.features))
    mean = np.broadcast_to(train_data.hist.mean(axis=0), test_data.hist.shape)
    out = {"l1_network": float(l1(pred, test_data.hist).mean()),
           "l1_nearest_neighbour": float(l1(nn, test_data.hist).mean()),
           "l1_training_mean": float(l1(mean, test_data.hist).mean()),
           "n_test": int(len(test_data.hist))}
    if noise_data is not None:
        out["l1_noise_floor"] = float(l1(noise_data.hist, test_data.hist).mean())
    return out, pred


def main(argv=None):
    """Full run: python -m paper_1703_09707_amd.surrogate [--train-sets 4096] ..."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser()
    ap.add_argument("--train-sets", type=int, default=4096)
    ap.add_argument("--test-sets", type=int, default=256)
    ap.add_argument("--rays", type=int, default=4096, help="rays per side of each map's lattice")
    ap.add_argument("--npix", type=int, default=512)
    ap.add_argument("--sigmas", type=int, default=4, help="Gaussian source sizes per map")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--precision", default="fp64_expansion",
                    help="how the maps are shot: fp64_expansion, fp32_bulk or fp64")
    ap.add_argument("--seed", type=int, default=W.BASE_SEED + 4)
    ap.add_argument("--out", default=None, help="write the JSON result here too")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    kw = dict(rays_per_side=a.rays, npix=a.npix, sigmas_per_map=a.sigmas, precision=a.precision, log=log)
    t0 = time.perf_counter()
    log("# training maps")
    train_data = generate(a.train_sets, a.seed, **kw)
    log("# held-out maps")
    test_rng = np.random.Generator(np.random.PCG64(a.seed + 1))
    test_params, _ = W.draw_batch_params(test_rng, a.test_sets)
    test_data = generate(a.test_sets, a.seed + 1, params=test_params, **kw)
    log("# held-out parameters again, other star fields (noise floor)")
    noise_data = generate(a.test_sets, a.seed + 1, params=test_params, star_seed_offset=500000, **kw)
    t_data = time.perf_counter() - t0
    log("# training")
    t1 = time.perf_counter()
    net, std, hist = train(train_data, steps=a.steps, batch=a.batch, lr=a.lr, log=log)
    t_train = time.perf_counter() - t1
    res, pred = evaluate(net, std, train_data, test_data, noise_data)
    torch = _torch()
    x = torch.from_numpy(std(test_data.features)).cuda()
    chunks = [x[i:i + net.max_batch].contiguous() for i in range(0, x.shape[0], net.max_batch)]
    for c in chunks:
        net.forward(c)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(20):
        for c in chunks:
            net.forward(c)
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t2) / 20
    res.update({
        "train_examples": int(len(train_data.hist)), "train_sets": a.train_sets, "test_sets": a.test_sets,
        "rays_per_map": a.rays ** 2, "map": [a.npix, a.npix], "sigmas_per_map": a.sigmas,
        "precision": a.precision, "steps": a.steps, "batch": a.batch,
        "loss_first_last": [hist[0][1], hist[-1][1]],
        "seconds_data": t_data, "seconds_shooting": train_data.seconds_shooting + test_data.seconds_shooting
        + noise_data.seconds_shooting, "seconds_train": t_train,
        "interactions": train_data.interactions + test_data.interactions + noise_data.interactions,
        "predict_us_per_example": 1e6 * t_pred / len(test_data.hist),
        "shoot_ms_per_map": 1e3 * test_data.seconds_shooting / a.test_sets,
    })
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    net.close()


if __name__ == "__main__":
    main()
