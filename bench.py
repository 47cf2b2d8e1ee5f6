"""Benchmark: backward ray shooting (arXiv:1703.09707, Algorithm 1) on one MI355X.

A step is one pass of Algorithm 1 over the whole workload: every ray of the
8192 x 8192 lattice through all 16384 stars, binned into the 1024 x 1024 map
(raysh_map, FP64).  Inputs (stars, map) are resident in device memory before
the timed region.  The FP32-bulk form is timed the same way and reported
beside it.

Metric: ray-star interactions per second (N_rays * N_stars / time), with
rays/s alongside.  The roofline object prices the FP64 kernel's algorithmic
FLOPs (10 per interaction: 2 subtractions, 2 multiplies and 1 add for r^2,
1 division, 2 multiply-adds for the accumulation) against the FP64 vector
peak; the kernel's own time comes from HIP events recorded on the stream the
kernel runs on.

Launch shapes come from the library's autotuner (raysh_autotune, and
raysh_autotune_batch for the batch), run before the timed regions; the
chosen shapes are reported.  Secondary sections are timed as the median of
five runs after a warm-up.

Also reported: the FP32-bulk form with its roofline against the non-packed
FP32 vector peak and its misbinned fraction ray by ray against FP64, the
64-set batch in one graph-captured persistent launch (against single
launches, with the FP32-bulk misbinned fraction per set), the FP32-bulk
misbinned fraction on the 262144-star precision-study subtile, the split
star sum on 4194304 stars x 256^2 rays (against one pass per ray), the
far-field expansion, light curves, the learned surrogate and the oracle on
the host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp32]
                       [--no-batch] [--no-precision] [--no-split]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 10
PROFILE = os.path.join(ROOT, "profiles", "shoot_fp64_kernel_plain-fp64-large.txt")
PROFILE_LC = os.path.join(ROOT, "profiles", "light_curve_track_kernel_light-curves-large.txt")
FP64_VECTOR_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# FP32 without packed instructions (the library is compiled without them) issues at the FP64 rate
FP32_VECTOR_PEAK_TFLOPS = 78.6
PROFILE_FP32 = os.path.join(ROOT, "profiles", "shoot_fp32_kernel_plain-fp64-large.txt")
METRIC = "Gray-star interactions/s and rays/s at 1 GPU (FP64 vs FP32-bulk), % vector peak"
HBM_PEAK_GBS = 8000.0              # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-set batch timing")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision study")
    ap.add_argument("--no-split", action="store_true", help="skip the many-stars/few-rays study")
    ap.add_argument("--no-expansion", action="store_true", help="skip the far-field expansion study")
    ap.add_argument("--no-light-curves", action="store_true", help="skip the light-curve timing")
    ap.add_argument("--no-lc-given-order", action="store_true",
                    help="time light curves in the track order only (not also in the given order)")
    ap.add_argument("--cpu-rays", type=int, default=1024, help="side of the oracle's ray sample (about 15 s)")
    ap.add_argument("--cpu-all-rays", type=int, default=2048,
                    help="side of the ray sample of the all-cores oracle run")
    ap.add_argument("--tile", default=None, help="FP64 tile cx,cy,share[,stars per group] (default: library's)")
    ap.add_argument("--tile32", default=None, help="FP32-bulk tile cx,cy,star_tile")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch shapes")
    ap.add_argument("--no-per-ray", action="store_true",
                    help="compare FP32-bulk with FP64 by maps only (no per-ray bins; for counter runs, so that "
                         "every dispatch of the map kernels at full size is a map)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: none, always timed)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate section")
    ap.add_argument("--surrogate-steps", type=int, default=20000, help="training steps of the surrogate section")
    ap.add_argument("--runs", type=int, default=5, help="runs per secondary timing (median reported)")
    ap.add_argument("--no-probe", action="store_true", help="skip the FMA-rate probe")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized buffer 3 times (the reference kernel for "
                         "scaling HBM byte counters)")
    return ap.parse_args()


def measured_traffic(workload_tag, profile=PROFILE, kernel="shoot_fp64_kernel"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    a kernel, or None when the kernel sources or the workload (launch shape)
    have changed since the counters were taken."""
    from paper_1703_09707_amd import rocprof_summary as RS
    s = RS.read_summary(profile)
    if not s or "traffic_bytes_per_launch" not in s:
        return None
    if s.get("source_sha256") != RS.source_hash(kernel) or s.get("workload") != workload_tag:
        return None
    return float(s["traffic_bytes_per_launch"])


# The FMA probe: 2048 workgroups of 256 threads, 8 chains of 16384 FMAs per
# thread (1.07e9 wave-level FMA instructions, 1.37e11 FLOP per launch).
PROBE_BLOCKS = 2048
PROBE_ITERS = 16384


def fma_probe_section(torch, raysh, runs, skip_fp32):
    """Plain FMA rate of the box at the clock it holds right after the FP64
    maps: the probe kernel issues nothing but independent FMAs, so its rate
    is the most the vector ALUs sustain here, beside the datasheet peak
    (78.6 TFLOP/s at 2.4 GHz).  Its results are exact, and are checked."""
    out = {"workload": f"{PROBE_BLOCKS} x 256 threads x 8 chains x {PROBE_ITERS} FMA",
           "wave_fma_instructions": PROBE_BLOCKS * 4 * 8 * PROBE_ITERS}
    flop = 2.0 * PROBE_BLOCKS * 256 * 8 * PROBE_ITERS
    lane = torch.arange(PROBE_BLOCKS * 256, device="cuda") % 64
    for prec in ("fp64",) + (() if skip_fp32 else ("fp32_bulk",)):
        buf = raysh.fma_probe(prec, PROBE_BLOCKS, PROBE_ITERS)
        want = (8 * (lane + PROBE_ITERS) + 28).to(buf.dtype)   # sum over chains i < 8 of (lane + i + iters)
        if not bool(torch.equal(buf, want)):
            raise RuntimeError(f"FMA probe ({prec}) returned wrong values")
        ms = []
        for _ in range(max(runs, 5)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            raysh.fma_probe(prec, PROBE_BLOCKS, PROBE_ITERS, out=buf)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        t = sorted(ms)[len(ms) // 2]
        tf = flop / (t * 1e-3) / 1e12
        out[prec] = {"kernel_ms": t, "tflops": tf, "frac_of_peak": tf / FP64_VECTOR_PEAK_TFLOPS,
                     "clock_ghz_if_every_cycle_issues": tf / FP64_VECTOR_PEAK_TFLOPS * 2.4}
    return out


def time_steps(torch, ctx, w, precision, counts, steps, warmup):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.map(w.rays, w.pix, precision, counts=counts)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        ctx.map(w.rays, w.pix, precision, counts=counts)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return wall, kernel_ms


def median_seconds(torch, fn, runs, warm=1):
    """Median wall time of fn() over `runs` runs after `warm` untimed ones,
    each bracketed by device synchronisations; returns (median, all)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], ts


def misbinned_lower_bound(a, b, n_rays):
    """Rays in a different pixel, at least: half the L1 distance of two maps
    plus half the change of the binned total, over the rays shot."""
    l1 = int((a.long() - b.long()).abs().sum())
    dn = abs(int(a.long().sum()) - int(b.long().sum()))
    return 0.5 * (l1 + dn) / n_rays


def batch_section(torch, raysh, W, runs, tune, cache):
    """64 parameter sets of uneven star counts in one persistent,
    graph-captured launch (replayed), against one single launch per set; the
    launch shape of each precision chosen by raysh_autotune_batch."""
    sets = W.batch_workloads()
    ctxs = [raysh.Context(x.lens) for x in sets]
    rays = [x.rays for x in sets]
    pix = [x.pix for x in sets]
    inter = sum(x.interactions for x in sets)
    n_rays = sum(x.rays.n_rays for x in sets)
    out = {"workload": "batch-64: 64 sets x 4096^2 rays, 512^2 maps, N* %d..%d" % (
        min(x.lens.n_stars for x in sets), max(x.lens.n_stars for x in sets)),
        "interactions": inter, "rays": n_rays, "runs": runs}
    maps = {}
    for prec in ("fp64", "fp32_bulk"):
        t0 = time.perf_counter()
        tile = raysh.autotune_batch(ctxs, rays, pix, prec, cache) if tune else ctxs[0].get_tile(prec)
        t_tune = time.perf_counter() - t0
        m = [torch.zeros((p.NY, p.NX), dtype=torch.int32, device="cuda") for p in pix]
        raysh.map_batch(ctxs, rays, pix, prec, counts=m)      # builds and captures the graph
        torch.cuda.synchronize()
        maps[prec] = [x.clone() for x in m]
        dt, all_t = median_seconds(torch, lambda: raysh.map_batch(ctxs, rays, pix, prec, counts=m), runs, warm=0)
        out[prec] = {"value": inter / dt, "unit": "interactions/s", "rays_per_s": n_rays / dt, "seconds": dt,
                     "seconds_all": all_t, "tile": list(tile), "tune_seconds": t_tune,
                     "roofline_frac": FLOP_PER_INTERACTION * inter / dt / 1e12 / (
                         FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS)}
    fr = [misbinned_lower_bound(a, b, x.rays.n_rays) for a, b, x in zip(maps["fp64"], maps["fp32_bulk"], sets)]
    out["fp32_bulk"]["misbinned_fraction_vs_fp64_per_set"] = {"max": max(fr), "mean": sum(fr) / len(fr),
                                                              "bound": "lower bound from each set's maps"}
    del maps

    def singles():
        for c, x, p in zip(ctxs, rays, pix):
            c.map(x, p, "fp64")
    single, all_t = median_seconds(torch, singles, runs)
    out["fp64_single_launches"] = {"value": inter / single, "unit": "interactions/s", "seconds": single,
                                   "seconds_all": all_t, "tile": list(ctxs[0].get_tile("fp64"))}
    out["speedup_vs_plain_fp64"] = {p: single / out[p]["seconds"] for p in ("fp64", "fp32_bulk")}
    for c in ctxs:
        c.close()
    return out


def precision_section(torch, raysh, W, runs):
    """FP32-bulk against FP64, ray by ray, on the central 2048^2 rays of the
    262144-star precision-study lattice."""
    w = W.precision_study()
    sub = W.precision_subtile(w, 2048)
    with raysh.Context(w.lens) as ctx:
        _, _, b64 = ctx.shoot(sub, "fp64", w.pix, beta=False)
        _, _, b32 = ctx.shoot(sub, "fp32_bulk", w.pix, beta=False)
        frac = float((b32 != b64).sum()) / b64.numel()
        c = torch.zeros((w.pix.NY, w.pix.NX), dtype=torch.int32, device="cuda")
        t32, _ = median_seconds(torch, lambda: ctx.map(sub, w.pix, "fp32_bulk", counts=c), runs)
        t64, _ = median_seconds(torch, lambda: ctx.map(sub, w.pix, "fp64", counts=c), runs)
    inter = sub.n_rays * w.lens.n_stars
    return {"workload": "precision-study subtile: 2048^2 rays x 262144 stars", "interactions": inter,
            "misbinned_fraction_fp32_bulk_vs_fp64": frac, "misbinned_kind": "per ray",
            "fp64_seconds": t64, "fp32_bulk_seconds": t32, "speedup": t64 / t32,
            "fp64_interactions_per_s": inter / t64, "fp32_bulk_interactions_per_s": inter / t32}


def split_section(torch, raysh, W, runs):
    """Many stars, few rays: 4194304 stars x 256^2 rays.  One pass per ray
    runs 16 workgroups; the split star sum spreads each ray's sum over
    workgroups (automatic part count)."""
    w = W.large_star_field(1 << 22, 256, 256)
    out = {"workload": "large-star-field: 4194304 Salpeter stars x 256^2 rays, 256^2 map",
           "interactions": w.interactions}
    with raysh.Context(w.lens) as ctx:
        for label, parts in (("split_auto", 0), ("one_pass", 1)):
            ctx.set_star_split(parts)
            counts = torch.zeros((w.pix.NY, w.pix.NX), dtype=torch.int32, device="cuda")
            dt, all_t = median_seconds(torch, lambda: ctx.map(w.rays, w.pix, "fp64", counts=counts), runs)
            out[label] = {"value": w.interactions / dt, "unit": "interactions/s", "seconds": dt,
                          "seconds_all": all_t}
    out["speedup"] = out["one_pass"]["seconds"] / out["split_auto"]["seconds"]
    return out


def expansion_section(torch, raysh, W, w, fp64_seconds, steps, warmup, runs):
    """FP64 with the far field of the star sum as local expansions, on the
    large configuration (time per map against the one-pass FP64 map, and the
    fraction of rays binned differently), and on the central 2048^2 rays of
    the 262144-star precision-study lattice."""
    out = {"workload": w.name, "interactions_equivalent": w.interactions}
    with raysh.Context(w.lens) as ctx:
        counts = torch.zeros((w.pix.NY, w.pix.NX), dtype=torch.int32, device="cuda")
        # a map takes under a millisecond: 200 untimed maps bring the clock
        # to the level a run of many maps (as the surrogate's) holds
        wall, kms = time_steps(torch, ctx, w, "fp64_expansion", counts, steps, max(warmup, 200))
        _, _, be = ctx.shoot(w.rays, "fp64_expansion", w.pix, beta=False)
        _, _, b64 = ctx.shoot(w.rays, "fp64", w.pix, beta=False)
        frac = float((be != b64).sum()) / be.numel()
        del be, b64
    out["large"] = {"ms_per_map": 1e3 * wall / steps, "kernel_ms": sum(kms) / len(kms),
                    "kernel_ms_median": sorted(kms)[len(kms) // 2],
                    "rays_per_s": w.rays.n_rays / (wall / steps),
                    "equivalent_interactions_per_s": w.interactions / (wall / steps),
                    "speedup_vs_fp64": fp64_seconds / (wall / steps),
                    "misbinned_fraction_vs_fp64": frac}
    p = W.precision_study()
    sub = W.precision_subtile(p, 2048)
    with raysh.Context(p.lens) as ctx:
        ctx.shoot(sub.block(0, 0, 256, 256), "fp64_expansion", p.pix, beta=False)   # builds the star cells
        _, _, be = ctx.shoot(sub, "fp64_expansion", p.pix, beta=False)
        _, _, b64 = ctx.shoot(sub, "fp64", p.pix, beta=False)
        frac = float((be != b64).sum()) / be.numel()
        c = torch.zeros((p.pix.NY, p.pix.NX), dtype=torch.int32, device="cuda")
        te, _ = median_seconds(torch, lambda: ctx.map(sub, p.pix, "fp64_expansion", counts=c), runs)
        t64, _ = median_seconds(torch, lambda: ctx.map(sub, p.pix, "fp64", counts=c), runs)
    out["precision_study_subtile"] = {"workload": "2048^2 rays x 262144 stars", "seconds": te,
                                      "fp64_seconds": t64, "speedup_vs_fp64": t64 / te,
                                      "misbinned_fraction_vs_fp64": frac}
    return out


def light_curve_section(torch, raysh, W, steps, given_order=True):
    """Light curves: the map of the large configuration seen by a Gaussian
    source of 2 pixels, then 2^20 straight tracks of 256 samples across it,
    visited in the library's track order, with the end points in that order
    (both computed once per track set).  The
    light-curve kernel is a gather bound by HBM: its algorithmic bytes are
    the curves written, the track end points read and the source map read
    once."""
    lw = W.light_curves_large()
    w = lw.maps
    norm = (w.rays.dx * w.rays.dy) / (w.pix.Px * w.pix.Py)
    with raysh.Context(w.lens) as ctx:
        counts = ctx.map(w.rays, w.pix, "fp64")
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731
    mu, grid = raysh.source_map(counts, w.pix, norm, lw.profile, lw.size)
    tracks = [torch.from_numpy(a).cuda() for a in W.light_curve_tracks(grid, lw.n_tracks, lw.length)]
    curves = torch.empty((lw.n_tracks, lw.n_samples), dtype=torch.float64, device="cuda")
    order, srt = raysh.track_order(grid, *tracks, sorted_end_points=True)
    for _ in range(100):   # steady clock: the kernel takes about half a millisecond
        raysh.light_curves(mu, grid, *tracks, lw.n_samples, out=curves, order=order, sorted=srt)
    torch.cuda.synchronize()
    sm, so, lc, lu = [], [], [], []
    for _ in range(steps):
        a, b, c, d, e = ev(), ev(), ev(), ev(), ev()
        a.record(stream)
        mu, grid = raysh.source_map(counts, w.pix, norm, lw.profile, lw.size)
        b.record(stream)
        order, srt = raysh.track_order(grid, *tracks, sorted_end_points=True)
        c.record(stream)
        raysh.light_curves(mu, grid, *tracks, lw.n_samples, out=curves, order=order, sorted=srt)
        d.record(stream)
        if given_order:
            raysh.light_curves(mu, grid, *tracks, lw.n_samples, out=curves)
        e.record(stream)
        torch.cuda.synchronize()
        sm.append(a.elapsed_time(b))
        so.append(b.elapsed_time(c))
        lc.append(c.elapsed_time(d))
        if given_order:
            lu.append(d.elapsed_time(e))
    med = lambda v: sorted(v)[len(v) // 2]   # noqa: E731
    lc_ms = med(lc)
    samples = lw.n_tracks * lw.n_samples
    nbytes = samples * 8 + lw.n_tracks * (32 + 4) + mu.numel() * 8   # curves, end points + order, map
    achieved = nbytes / (lc_ms * 1e-3) / 1e9
    return {"workload": lw.name, "samples": samples,
            "source_map_ms": med(sm),
            "track_order_ms": med(so),
            "light_curve_kernel_ms": lc_ms,
            "light_curve_kernel_ms_given_order": med(lu) if lu else None,
            "timing": f"median of {len(lc)} runs (HIP events) after 100 untimed launches",
            "samples_per_s": samples / (lc_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "kernel": "light_curve_track_kernel",
                         "bytes_per_launch": nbytes,
                         "traffic": measured_traffic("light-curves-large 2^20 tracks x 256 samples, track order",
                                                     PROFILE_LC, "light_curve_track_kernel")}}


def surrogate_section(steps):
    """The learned part at its full size: 4096 shooter-generated 512^2 maps
    (4096^2 rays each, FP64 with the far field expanded) over sampled
    (kappa, gamma, kappa_*/kappa), four Gaussian sources per map; the
    network trained on them by the library's kernels; evaluated on 256
    held-out sets against the mean of four star-field realisations each;
    out-of-domain queries answered by the plain FP64 shooter."""
    from paper_1703_09707_amd import surrogate as S

    def log(msg):
        if not msg.startswith("  "):
            print(msg, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = S.run(steps=steps, log=log)
    res["seconds_total"] = time.perf_counter() - t0
    res["workload"] = ("surrogate: 4096 training maps of 512^2 pixels (4096^2 rays each), 4 Gaussian sources "
                       "per map, 3-layer MLP (width 256, BF16 weights, FP32 accumulation), 64-bin "
                       "log-magnification histograms, 256 held-out sets")
    return res


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, side):
    """The oracle, as it stands, on the central side x side rays."""
    from oracle import shooter as ora
    blk = w.rays.block((w.rays.nx - side) // 2, (w.rays.ny - side) // 2, side, side)
    t0 = time.perf_counter()
    ora.map_counts(w.lens.as_tuple(), blk.as_tuple(), w.pix.as_tuple())
    dt = time.perf_counter() - t0
    inter = blk.n_rays * w.lens.n_stars
    return {"value": inter / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "rays_per_s": blk.n_rays / dt,
            "sample": f"central {side}x{side} rays of the 8192^2 lattice x {w.lens.n_stars} stars "
                      f"({inter:.3e} interactions, {dt:.1f} s, single thread)"}


def _oracle_band(job):
    from oracle import shooter as ora
    lens, rays, pix = job
    ora.map_counts(lens, rays, pix)
    return rays[5]


def _ready(_):
    return os.getpid()


def cpu_parallel_baseline(w, side, procs):
    """The oracle as it stands, run as `procs` independent processes on
    disjoint row bands of the central side x side rays (band additivity makes
    the bands' maps add up to the block's map exactly).  Runs before the GPU
    is touched, so the workers are plain forks of a CPU-only process."""
    import multiprocessing as mp
    blk = w.rays.block((w.rays.nx - side) // 2, (w.rays.ny - side) // 2, side, side)
    edges = [side * k // procs for k in range(procs + 1)]
    jobs = [(w.lens.as_tuple(), blk.block(0, edges[k], side, edges[k + 1] - edges[k]).as_tuple(),
             w.pix.as_tuple()) for k in range(procs)]
    with mp.get_context("fork").Pool(procs) as pool:
        pool.map(_ready, range(procs), chunksize=1)   # workers are up before the clock starts
        t0 = time.perf_counter()
        done = pool.map(_oracle_band, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    assert sum(done) == side
    inter = side * side * w.lens.n_stars
    return {"value": inter / dt, "unit": "interactions/s", "cores": procs, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"central {side}x{side} rays of the 8192^2 lattice x {w.lens.n_stars} stars in "
                      f"{procs} row bands, one process each ({inter:.3e} interactions, {dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU form "
              "(ray-band sharding plus an int32 map reduce) is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1703_09707_amd import raysh
    from paper_1703_09707_amd import workloads as W

    cpu_all = None
    if not args.no_cpu:   # before anything initialises the GPU: the pool forks this process
        procs = max(1, min(16, os.cpu_count() or 1))
        print(f"# cpu baseline, all cores ({procs} processes)", file=sys.stderr, flush=True)
        cpu_all = cpu_parallel_baseline(W.plain_fp64_large(), args.cpu_all_rays, procs)

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    w = W.plain_fp64_large()
    inter = w.interactions
    ctx = raysh.Context(w.lens, device=0)
    if args.tile:
        t = [int(v) for v in args.tile.split(",")]
        ctx.set_tile("fp64", t[0], t[1], share=t[2], star_tile=t[3] if len(t) > 3 else 0)
    if args.tile32:
        cx, cy, st = (int(v) for v in args.tile32.split(","))
        ctx.set_tile("fp32_bulk", cx, cy, star_tile=st)
    tuning = {}
    for prec, given in (("fp64", args.tile), ("fp32_bulk", args.tile32)):
        if given or args.no_tune:
            tuning[prec] = {"tile": list(ctx.get_tile(prec)), "chosen_by": "given" if given else "library default"}
            continue
        print(f"# autotune {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        t = ctx.autotune(w.rays, w.pix, prec, cache_path=args.tune_cache)
        tuning[prec] = {"tile": list(t), "chosen_by": "raysh_autotune", "seconds": time.perf_counter() - t0}
    counts = torch.zeros((w.pix.NY, w.pix.NX), dtype=torch.int32, device="cuda")

    print(f"# fp64: {args.steps} steps after {args.warmup} warmup", file=sys.stderr, flush=True)
    wall, kms = time_steps(torch, ctx, w, "fp64", counts, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    k_avg = sum(kms) / len(kms)
    achieved = FLOP_PER_INTERACTION * inter / (k_avg * 1e-3) / 1e12
    tile = ctx.get_tile("fp64")
    tag = "plain-fp64-large tile %d,%d,%d,%d" % tile

    out = {
        "metric": METRIC,
        "value": inter / (wall / args.steps),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded star field, Salpeter masses)",
        "config": {"workload": "plain-fp64-large", "n_stars": w.lens.n_stars,
                   "rays": [w.rays.nx, w.rays.ny], "map": [w.pix.NX, w.pix.NY],
                   "kappa_star": w.lens.kappa_star, "kappa_c": w.lens.kappa_c,
                   "gamma": [w.lens.gamma1, w.lens.gamma2],
                   "tile_fp64": list(tile)},
        "tuning": tuning,
        "rays_per_s": w.rays.n_rays / (wall / args.steps),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(tag), "kernel": "shoot_fp64_kernel",
                     "kernel_ms": k_avg,
                     "flop_per_launch": FLOP_PER_INTERACTION * inter},
    }
    if not args.no_probe:
        print("# FMA probe", file=sys.stderr, flush=True)
        out["fma_probe"] = fma_probe_section(torch, raysh, args.runs, args.no_fp32)
        # the shooter against the FMA rate this machine sustains at its clock under load
        out["roofline"]["frac_of_fma_probe"] = achieved / out["fma_probe"]["fp64"]["tflops"]
    if not args.no_fp32:
        print("# fp32_bulk", file=sys.stderr, flush=True)
        c32 = torch.zeros_like(counts)
        wall32, kms32 = time_steps(torch, ctx, w, "fp32_bulk", c32, args.steps, args.warmup)
        k32 = sum(kms32) / len(kms32)
        ach32 = FLOP_PER_INTERACTION * inter / (k32 * 1e-3) / 1e12
        tile32 = ctx.get_tile("fp32_bulk")
        m64 = ctx.map(w.rays, w.pix, "fp64")
        m32 = ctx.map(w.rays, w.pix, "fp32_bulk")
        lower = misbinned_lower_bound(m64, m32, w.rays.n_rays)
        del m64, m32
        per_ray = None
        if not args.no_per_ray:
            _, _, b64 = ctx.shoot(w.rays, "fp64", w.pix, beta=False)
            _, _, b32 = ctx.shoot(w.rays, "fp32_bulk", w.pix, beta=False)
            per_ray = float((b64 != b32).sum()) / w.rays.n_rays
            del b64, b32
        out["fp32_bulk"] = {
            "value": inter / (wall32 / args.steps), "unit": "interactions/s",
            "rays_per_s": w.rays.n_rays / (wall32 / args.steps),
            "ms_per_step": 1e3 * wall32 / args.steps, "kernel_ms": k32,
            "speedup_vs_fp64": wall / wall32,
            "misbinned_fraction_vs_fp64": per_ray,
            "misbinned_kind": "per ray, every ray of the 8192^2 lattice against the FP64 path's bins",
            "misbinned_fraction_lower_bound_from_maps": lower,
            "tile": list(tile32),
            "roofline": {"bound": "alu", "achieved": ach32, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach32 / FP32_VECTOR_PEAK_TFLOPS, "kernel": "shoot_fp32_kernel",
                         "peak_note": "FP32 vector peak without packed instructions (the library is compiled "
                                      "without them); 157.3 TFLOP/s with them",
                         "traffic": measured_traffic("plain-fp64-large tile32 %d,%d,%d,%d" % tile32,
                                                     PROFILE_FP32, "shoot_fp32_kernel"),
                         "kernel_ms": k32, "flop_per_launch": FLOP_PER_INTERACTION * inter}}
        if "fma_probe" in out and "fp32_bulk" in out["fma_probe"]:
            out["fp32_bulk"]["roofline"]["frac_of_fma_probe"] = ach32 / out["fma_probe"]["fp32_bulk"]["tflops"]
    ctx.close()
    del counts
    # end to end, as the paper times a map: context and star upload, one map,
    # the map back on the host (into a pinned buffer the caller keeps)
    host_map = torch.empty((w.pix.NY, w.pix.NX), dtype=torch.int32, pin_memory=True)
    host_map.copy_(torch.zeros((w.pix.NY, w.pix.NX), dtype=torch.int32, device="cuda"))   # its first use
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = raysh.Context(w.lens, device=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m = ctx.map(w.rays, w.pix, "fp64")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    host_map.copy_(m)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ctx.close()
    out["end_to_end_ms"] = {"init_and_star_upload": 1e3 * (t1 - t0), "map": 1e3 * (t2 - t1),
                            "map_to_host": 1e3 * (t3 - t2), "total": 1e3 * (t3 - t0)}
    del m, host_map
    if not args.no_batch:
        print("# batch (64 sets)", file=sys.stderr, flush=True)
        out["batch"] = batch_section(torch, raysh, W, args.runs, not args.no_tune, args.tune_cache)
    if not args.no_precision:
        print("# precision study", file=sys.stderr, flush=True)
        out["precision_study"] = precision_section(torch, raysh, W, args.runs)
    if not args.no_split:
        print("# many stars, few rays (split star sum)", file=sys.stderr, flush=True)
        out["split_star_sum"] = split_section(torch, raysh, W, args.runs)
    if not args.no_expansion:
        print("# far-field expansion", file=sys.stderr, flush=True)
        out["fp64_expansion"] = expansion_section(torch, raysh, W, w, wall / args.steps, args.steps,
                                                  args.warmup, args.runs)
    if not args.no_light_curves:
        print("# light curves", file=sys.stderr, flush=True)
        out["light_curves"] = light_curve_section(torch, raysh, W, max(args.steps, args.runs),
                                                  not args.no_lc_given_order)
    if not args.no_surrogate:
        print("# learned surrogate", file=sys.stderr, flush=True)
        out["surrogate"] = surrogate_section(args.surrogate_steps)
    if not args.no_cpu:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_rays)
        out["cpu_baseline_all_cores"] = cpu_all
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
