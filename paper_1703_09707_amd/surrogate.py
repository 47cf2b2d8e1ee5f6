"""Learned surrogate for magnification histograms (binding and host driver).

The Bayesian Monte Carlo analysis that motivates fast map generation
(arXiv:1703.09707, Sec. 1) needs the magnification statistics of many lens
parameter sets.  Here the shooter generates maps over sampled
(kappa, gamma, kappa_*/kappa); each map, seen by Gaussian sources of several
sizes, gives a 64-bin histogram of log10(mu_sigma / mu_macro); a small network
(4 -> 256 -> 256 -> 64, BF16 weights, FP32 accumulation) learns to predict
the histogram from (kappa, gamma, kappa_*/kappa, log10 sigma).  The shooter
remains the reference: held-out histograms are compared by L1 distance with the
network's predictions, with the realisation-noise floor (two star fields at
the same parameters) and with a no-network baseline (the nearest training
example in standardised feature space).

Queries go through ``Surrogate``: a query whose standardised features lie
inside the training data's box and near a training example is answered by
the network; any other query is answered by shooting its map and taking its
histogram (the plain shooter as fallback), so the surrogate never
extrapolates.  The held-out evaluation compares with the mean histogram of
several star-field realisations per parameter set, so that it measures the
network's error and not the scatter of one realisation.

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
    pool = []   # one context per set of a chunk, given each chunk's lenses (raysh_set_lens)
    try:
        for c0 in range(0, len(params), chunk):
            part = params[c0:c0 + chunk]
            grids = []
            for s, p in enumerate(part):
                srng = np.random.Generator(np.random.PCG64(seed + star_seed_offset + 1000 + c0 + s))
                m = W.salpeter_masses(p["n_stars"], srng)
                x, y, _ = W.star_field(m, p["kappa_star"], srng)
                lens = (p["kappa_c"], p["gamma"], 0.0, x, y, m)
                if s < len(pool):
                    pool[s].set_lens(lens)
                else:
                    pool.append(R.Context(lens, device=device))
                grids.append(W.centred_rays(p["hx"], p["hy"], rays_per_side, rays_per_side))
                inter += rays_per_side ** 2 * p["n_stars"]
                rays += rays_per_side ** 2
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctxs = pool[:len(part)]
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
            if log:
                log(f"  shot sets {c0}..{c0 + len(part) - 1} ({t_shoot:.1f} s shooting)")
    finally:
        for c in pool:
            c.close()
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
    g = torch.Generator(device=X.device).manual_seed(seed)   # minibatches drawn on the GPU
    n = X.shape[0]
    hist = []
    for step in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g, device=X.device)
        xb, yb = X[idx].contiguous(), Y[idx].contiguous()
        rate = lr * 0.5 * (1 + math.cos(math.pi * step / steps))   # cosine decay
        loss = net.train_step(xb, yb, rate)
        if step % 200 == 0 or step == steps - 1:
            hist.append((step, float(loss.item())))
            if log:
                log(f"  step {step} loss {hist[-1][1]:.4f}")
    return net, std, hist


# ----------------------------------------------------------------- one parameter set, shot
@dataclasses.dataclass
class ShooterConfig:
    """How the fallback (and the data) shoot a parameter set: a square
    lattice of rays_per_side^2 rays over the preimage box of a window of
    `window` x `window` Einstein angles binned into npix^2 pixels."""
    rays_per_side: int = 4096
    npix: int = 512
    window: float = 10.0
    precision: str = "fp64"
    max_stars: int = 1 << 21


def lens_for(kappa, gamma, f, window, rng, max_stars=1 << 21):
    """The lens of one parameter set, drawn as the data are (workloads.
    draw_batch_params): kappa_* = f kappa, kappa_c = kappa - kappa_*,
    gamma2 = 0, a disk of radius 1.2 x the preimage box's half diagonal
    holding N* = round(kappa_* R^2 / <m>) Salpeter stars.  Returns
    (lens tuple, hx, hy).  ValueError for parameters the shooter cannot
    answer: not finite, kappa outside [0, 2), f outside [0, 1], gamma < 0,
    a macro lens within 1e-3 of critical (|det A| < 1e-3), or more than
    max_stars stars."""
    vals = (kappa, gamma, f)
    if not all(math.isfinite(v) for v in vals):
        raise ValueError(f"parameters not finite: {vals}")
    if not (0.0 <= kappa < 2.0 and 0.0 <= f <= 1.0 and gamma >= 0.0):
        raise ValueError(f"parameters outside the shooter's range: kappa {kappa}, gamma {gamma}, f {f}")
    det = (1 - kappa) ** 2 - gamma ** 2
    if abs(det) < 1e-3:
        raise ValueError(f"macro lens too close to critical: |det A| = {abs(det):.2e}")
    hx, hy = W.preimage_half_widths(kappa, gamma, 0.0, window / 2, window / 2)
    radius = 1.2 * math.hypot(hx, hy)
    ks = f * kappa
    n = int(round(ks * radius ** 2 / W.salpeter_mean()))
    if n > max_stars:
        raise ValueError(f"{n} stars exceed the fallback's limit of {max_stars}")
    m = W.salpeter_masses(n, rng)
    x, y, _ = W.star_field(m, ks, rng) if n > 0 else (np.zeros(0), np.zeros(0), None)
    return (kappa - ks, gamma, 0.0, x, y, m), hx, hy


def shoot_histograms(features, cfg: ShooterConfig, seed, device=0):
    """The shooter's histograms for rows of raw features (kappa, gamma, f,
    log10 sigma): one map per row (star field seeded by seed + row), seen by
    a Gaussian source of width sigma.  ValueError for a row the shooter
    cannot answer (see lens_for; also a source too large for the map)."""
    torch = _torch()
    feats = np.atleast_2d(np.asarray(features, np.float64))
    pix = W.centred_window(cfg.window, cfg.npix)
    hist = Histogrammer(cfg.npix, cfg.npix, device)
    out = np.empty((len(feats), N_BINS), np.float32)
    for r, (kappa, gamma, f, lsig) in enumerate(feats):
        sigma = 10.0 ** lsig
        if not (math.isfinite(sigma) and 0.0 < 3.0 * sigma < 0.5 * cfg.window):
            raise ValueError(f"source width {sigma} does not fit the {cfg.window} x {cfg.window} window")
        rng = np.random.Generator(np.random.PCG64(seed + r))
        lens, hx, hy = lens_for(kappa, gamma, f, cfg.window, rng, cfg.max_stars)
        grid = W.centred_rays(hx, hy, cfg.rays_per_side, cfg.rays_per_side)
        with R.Context(lens, device=device) as ctx:
            counts = ctx.map(grid, pix, cfg.precision)
        norm = (grid.dx * grid.dy) / (pix.Px * pix.Py)
        _, h = hist(counts, norm, sigma, pix.Px, pix.Py, W.mean_magnification(kappa, gamma, 0.0))
        out[r] = h.cpu().numpy()
    return out


def predict(net: MLP, std: Standardiser, features):
    torch = _torch()
    x = torch.from_numpy(std(np.asarray(features, np.float32))).to(f"cuda:{net.device}")
    out = []
    for i in range(0, x.shape[0], net.max_batch):
        out.append(net.forward(x[i:i + net.max_batch].contiguous()))
    return torch.cat(out).cpu().numpy()


def evaluate(net, std, train_data: Dataset, test_data: Dataset, noise_data: Dataset | None = None,
             realisations=()):
    """Held-out L1 of the network, of the nearest-neighbour baseline and of
    the training-mean histogram against the held-out histograms.

    test_data holds one star-field realisation per held-out set; the
    `realisations` (more Datasets of the same sets and sources, other star
    fields) join it in the target, which is then the mean histogram of all
    of them (so the evaluation measures the network's error rather than the
    scatter of one realisation).  noise_data, one more independent
    realisation, gives the realisation-noise floor: its L1 to the same
    target."""
    runs = [test_data, *realisations]
    for d in runs[1:]:
        assert np.array_equal(d.features, test_data.features), "realisations of other sets or sources"
    target = np.mean([d.hist.astype(np.float64) for d in runs], axis=0)
    pred = predict(net, std, test_data.features)
    nn = nearest_neighbour(std(train_data.features), train_data.hist, std(test_data.features))
    mean = np.broadcast_to(train_data.hist.mean(axis=0), test_data.hist.shape)
    out = {"l1_network": float(l1(pred, target).mean()),
           "l1_nearest_neighbour": float(l1(nn, target).mean()),
           "l1_training_mean": float(l1(mean, target).mean()),
           "realisations_per_target": len(runs),
           "n_test": int(len(test_data.hist))}
    if noise_data is not None:
        out["l1_noise_floor"] = float(l1(noise_data.hist, target).mean())
    return out, pred


@dataclasses.dataclass
class Domain:
    """Where the network may answer: standardised features inside the
    training data's box and no farther from a training example than
    `radius` (twice the 99th percentile of the training examples' own
    nearest-neighbour distances)."""
    lo: np.ndarray
    hi: np.ndarray
    radius: float
    points: np.ndarray

    @classmethod
    def fit(cls, xs):
        xs = np.asarray(xs, np.float64)
        d = _nn_distances(xs, xs, exclude_self=True)
        return cls(xs.min(axis=0), xs.max(axis=0), 2.0 * float(np.quantile(d, 0.99)), xs)

    def contains(self, xs):
        xs = np.atleast_2d(np.asarray(xs, np.float64))
        inside = np.all((xs >= self.lo) & (xs <= self.hi), axis=1) & np.all(np.isfinite(xs), axis=1)
        near = np.zeros(len(xs), bool)
        if inside.any():
            near[inside] = _nn_distances(xs[inside], self.points) <= self.radius
        return inside & near


def _nn_distances(q, pts, exclude_self=False, chunk=2048):
    """Distance from each row of q to its nearest row of pts."""
    out = np.empty(len(q))
    for i in range(0, len(q), chunk):
        d = ((q[i:i + chunk, None, :] - pts[None, :, :]) ** 2).sum(-1)
        if exclude_self:
            d[np.arange(d.shape[0]), np.arange(i, i + d.shape[0])] = np.inf
        out[i:i + chunk] = np.sqrt(d.min(axis=1))
    return out


class Surrogate:
    """The trained network with its domain, and the shooter behind it.

    query(features) answers rows inside the domain with the network and
    every other row by shooting it (shoot_histograms with `cfg`): the plain
    shooter is the fallback.  Returns (histograms [n, 64], source per row:
    "network" or "shooter")."""

    def __init__(self, net: MLP, std: Standardiser, train_data: Dataset, cfg: ShooterConfig | None = None,
                 seed=W.BASE_SEED + 9):
        self.net, self.std, self.cfg, self.seed = net, std, cfg or ShooterConfig(), seed
        self.domain = Domain.fit(std(train_data.features))

    def in_domain(self, features):
        return self.domain.contains(self.std(np.atleast_2d(np.asarray(features, np.float32))))

    def query(self, features):
        feats = np.atleast_2d(np.asarray(features, np.float64))
        ok = self.in_domain(feats)
        out = np.empty((len(feats), N_BINS), np.float32)
        if ok.any():
            out[ok] = predict(self.net, self.std, feats[ok])
        if (~ok).any():
            out[~ok] = shoot_histograms(feats[~ok], self.cfg, self.seed, self.net.device)
        return out, np.where(ok, "network", "shooter")


def run(train_sets=4096, test_sets=256, rays=4096, npix=512, sigmas=4, steps=20000, batch=256, lr=2e-3,
        precision="fp64_expansion", seed=W.BASE_SEED + 4, realisations=4, log=None):
    """The whole learned part at a given size: shoot the training maps and
    the held-out maps (`realisations` star fields per held-out set, plus one
    more for the noise floor), train, evaluate, time the network against the
    shooter and answer out-of-domain queries through the fallback.  Returns
    a dict of results."""
    torch = _torch()
    log = log or (lambda msg: None)
    kw = dict(rays_per_side=rays, npix=npix, sigmas_per_map=sigmas, precision=precision, log=log)
    t0 = time.perf_counter()
    log("# training maps")
    train_data = generate(train_sets, seed, **kw)
    log("# held-out maps")
    test_rng = np.random.Generator(np.random.PCG64(seed + 1))
    test_params, _ = W.draw_batch_params(test_rng, test_sets)
    runs = [generate(test_sets, seed + 1, params=test_params, star_seed_offset=500000 * k, **kw)
            for k in range(realisations)]
    log("# held-out parameters again, another star field (noise floor)")
    noise_data = generate(test_sets, seed + 1, params=test_params, star_seed_offset=500000 * realisations, **kw)
    t_data = time.perf_counter() - t0
    log("# training")
    t1 = time.perf_counter()
    net, std, hist = train(train_data, steps=steps, batch=batch, lr=lr, log=log)
    t_train = time.perf_counter() - t1
    res, pred = evaluate(net, std, train_data, runs[0], noise_data, realisations=runs[1:])
    single, _ = evaluate(net, std, train_data, runs[0])
    x = torch.from_numpy(std(runs[0].features)).cuda()
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
    # the fallback: queries outside the training domain are shot
    sur = Surrogate(net, std, train_data, ShooterConfig(rays_per_side=rays, npix=npix, precision="fp64"))
    inside = sur.in_domain(runs[0].features)
    outside = np.array([[0.9, 0.05, 0.5, -1.0], [0.3, 0.75, 0.4, -0.5], [0.5, 0.3, 0.6, 0.1]])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _, src = sur.query(outside)
    torch.cuda.synchronize()
    t_fb = (time.perf_counter() - t3) / len(outside)
    res.update({
        "l1_against_one_realisation": {k: single[k] for k in ("l1_network", "l1_nearest_neighbour",
                                                               "l1_training_mean")},
        "train_examples": int(len(train_data.hist)), "train_sets": train_sets, "test_sets": test_sets,
        "rays_per_map": rays ** 2, "map": [npix, npix], "sigmas_per_map": sigmas,
        "precision": precision, "steps": steps, "batch": batch,
        "loss_first_last": [hist[0][1], hist[-1][1]],
        "seconds_data": t_data, "seconds_shooting": train_data.seconds_shooting + sum(
            d.seconds_shooting for d in runs) + noise_data.seconds_shooting, "seconds_train": t_train,
        "interactions": train_data.interactions + sum(d.interactions for d in runs) + noise_data.interactions,
        "predict_us_per_example": 1e6 * t_pred / len(runs[0].hist),
        "shoot_ms_per_map": 1e3 * runs[0].seconds_shooting / test_sets,
        "held_out_in_domain": float(inside.mean()),
        "fallback": {"queries": outside.tolist(), "answered_by": src.tolist(),
                     "ms_per_query": 1e3 * t_fb, "precision": "fp64"},
    })
    net.close()
    return res


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
    ap.add_argument("--realisations", type=int, default=4,
                    help="star fields per held-out set averaged into the evaluation's target")
    ap.add_argument("--seed", type=int, default=W.BASE_SEED + 4)
    ap.add_argument("--out", default=None, help="write the JSON result here too")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    res = run(a.train_sets, a.test_sets, a.rays, a.npix, a.sigmas, a.steps, a.batch, a.lr, a.precision, a.seed,
              a.realisations, log)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
