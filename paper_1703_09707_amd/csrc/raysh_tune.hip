// Launch-shape autotuner: times every compiled tile shape of one precision
// on a sample of the caller's work and keeps the fastest.  raysh_autotune
// times the one-shot kernels on a central sample of one ray block;
// raysh_autotune_batch times the persistent batch kernel on a sample batch
// (a central block of every set's rays).  Choices are cached in a plain text
// file, one line per key:
//   <arch> <cus> <hip runtime version> <kind> <precision> <log2 stars bucket>
//   <cx> <cy> <share> <star_tile> <ms>
// kind is "single" or "batch"; for a batch the bucket is that of the mean
// star count of its sets.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "raysh_ctx.h"

using raysh::ShootParams;
using raysh::TileShape;

namespace {

struct Key {
    std::string arch;
    int cus = 0;
    int runtime = 0;   // hipRuntimeGetVersion
    std::string kind;
    int precision = 0;
    int bucket = 0;
};

int star_bucket(int64_t n) {
    int b = 0;
    while ((int64_t(1) << b) <= n && b < 62) ++b;
    return b;
}

bool cache_lookup(const char *path, const Key &k, TileShape &t) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], arch[128], kind[32];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int cus, rt, prec, bucket, cx, cy, share, st;
        double ms;
        if (std::sscanf(line, "%127s %d %d %31s %d %d %d %d %d %d %lf", arch, &cus, &rt, kind, &prec, &bucket, &cx,
                        &cy, &share, &st, &ms) != 11)
            continue;   // a line of another format
        if (k.arch == arch && k.cus == cus && k.runtime == rt && k.kind == kind && k.precision == prec &&
            k.bucket == bucket) {
            t = TileShape{cx, cy, share, st};
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const Key &k, const TileShape &t, double ms) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %s %d %d %d %d %d %d %.4f\n", k.arch.c_str(), k.cus, k.runtime, k.kind.c_str(),
                 k.precision, k.bucket, t.cx, t.cy, t.share, t.star_tile, ms);
    std::fclose(f);
}

int make_key(int device, int precision, const char *kind, int64_t n_stars, Key &key) {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_error(e, "raysh_autotune");
    key.arch = prop.gcnArchName;
    for (char &c : key.arch)
        if (c == ' ') c = '_';
    key.cus = prop.multiProcessorCount;
    if (hipRuntimeGetVersion(&key.runtime) != hipSuccess) {
        (void)hipGetLastError();
        key.runtime = 0;
    }
    key.kind = kind;
    key.precision = precision;
    key.bucket = star_bucket(n_stars);
    return RAYSH_OK;
}

bool supported(int precision, const TileShape &t) {
    return precision == RAYSH_FP64 ? raysh::fp64_shape_supported(t) : raysh::fp32_shape_supported(t);
}

int shape_list(int precision, TileShape (&shapes)[32]) {
    const int n = precision == RAYSH_FP64 ? raysh::fp64_shape_list(shapes, 32) : raysh::fp32_shape_list(shapes, 32);
    return std::min(n, 32);
}

struct Timed {
    TileShape shape;
    double cost;
};

// Time `run` for every compiled shape: one warm-up, then the median of three
// launches timed by HIP events on `stream`; `cost` turns a shape and its
// median time into the figure to minimise.  Every shape's figure goes to
// `out`, the best first.  Returns a RAYSH_* code.
template <class Run, class Cost>
int time_shapes(int precision, hipStream_t stream, Run run, Cost cost, std::vector<Timed> &out) {
    TileShape shapes[32];
    const int n_shapes = shape_list(precision, shapes);
    hipEvent_t ev[4];
    for (auto &x : ev) (void)hipEventCreate(&x);
    int code = RAYSH_OK;
    out.clear();
    for (int i = 0; i < n_shapes && code == RAYSH_OK; ++i) {
        const TileShape &t = shapes[i];
        hipError_t e = run(t);   // warm-up
        float ms[3] = {0, 0, 0};
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(ev[rep], stream);
            if (e == hipSuccess) e = run(t);
            if (e == hipSuccess) e = hipEventRecord(ev[rep + 1], stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[rep + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms[rep], ev[rep], ev[rep + 1]);
        }
        if (e != hipSuccess) {
            code = hip_error(e, "raysh_autotune");
            break;
        }
        std::sort(ms, ms + 3);
        out.push_back(Timed{t, cost(t, ms[1])});
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    std::stable_sort(out.begin(), out.end(), [](const Timed &a, const Timed &b) { return a.cost < b.cost; });
    if (code == RAYSH_OK && out.empty()) code = set_error(RAYSH_EINVAL, "raysh_autotune: no compiled shape");
    return code;
}

void report(const TileShape &best, int *cx, int *cy, int *share, int *star_tile) {
    if (cx) *cx = best.cx;
    if (cy) *cy = best.cy;
    if (share) *share = best.share;
    if (star_tile) *star_tile = best.star_tile;
}

// Interactions per timed sample: long enough (about 20 ms at the FP64 rate)
// that the launch and the queue ramp are a small part of it.
constexpr double kSampleWork = 1e11;

// Shapes whose predicted time is within kFinalSpread of the best (at most
// kFinalists of them) are timed on the whole block when the best prediction
// is at most kFinalMaxMs.
constexpr int kFinalists = 3;
constexpr double kFinalSpread = 0.06;
constexpr double kFinalMaxMs = 500.0;

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The sample of one shape for raysh_autotune: whole tiles, in whole rounds
// of the workgroups the device holds at once (one round at least, more
// until about kSampleWork interactions or the block's own rounds), so that
// neither ragged tiles nor a part-filled last round bias the comparison.
// Returns the block's tile count through n_tiles and the sample's rounds.
raysh_rays shape_sample(const raysh_rays &r, const TileShape &t, int64_t n_stars, int64_t resident,
                        int64_t &n_tiles, int64_t &rounds) {
    const int64_t tw = raysh::tile_width(t), th = raysh::tile_height(t);
    const int64_t tiles_x = ceil_div(r.nx, tw), tiles_y = ceil_div(r.ny, th);
    n_tiles = tiles_x * tiles_y;
    const double round_work = (double)resident * tw * th * (double)std::max<int64_t>(n_stars, 1);
    int64_t want_rounds = std::max<int64_t>(1, (int64_t)std::ceil(kSampleWork / round_work));
    want_rounds = std::min<int64_t>(want_rounds, ceil_div(n_tiles, resident));
    const int64_t want = std::min<int64_t>(n_tiles, want_rounds * resident);
    const int64_t sx = std::min<int64_t>(tiles_x, want);
    const int64_t sy = std::min<int64_t>(tiles_y, std::max<int64_t>(1, want / sx));
    raysh_rays s = r;
    s.nx = std::min<int64_t>(r.nx, sx * tw);
    s.ny = std::min<int64_t>(r.ny, sy * th);
    s.i0 = r.i0 + (r.nx - s.nx) / 2;
    s.j0 = r.j0 + (r.ny - s.ny) / 2;
    rounds = ceil_div(sx * sy, resident);
    return s;
}

}  // namespace

extern "C" int raysh_autotune(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix,
                              int precision, const char *cache_path, int *cx, int *cy, int *share,
                              int *star_tile) {
    if (int r = validate_rays(rays)) return r;
    if (int r = validate_pixels(pix)) return r;
    if (int r = validate_tiled_precision(precision)) return r;
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", ctx->device);

    Key key;
    if (int r = make_key(ctx->device, precision, "single", ctx->n_stars, key)) return r;
    if (!cache_path) cache_path = std::getenv("RAYSH_AUTOTUNE_CACHE");

    TileShape best{};
    double best_ms = -1;
    const bool cached = cache_path && cache_lookup(cache_path, key, best) && supported(precision, best);
    if (!cached) {
        if (rays->nx == 0 || rays->ny == 0) return set_error(RAYSH_EINVAL, "raysh_autotune: empty ray block");
        int32_t *scratch = nullptr;
        const size_t map_bytes = (size_t)pix->nx * (size_t)pix->ny * 4;
        hipError_t e = hipMalloc(&scratch, map_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(RAYSH_ENOMEM, "raysh_autotune: scratch map");
        }
        // per shape: a sample of whole rounds; the figure compared is the
        // predicted time of the whole block, rounds(block) x time per round
        TileShape cur{};
        ShootParams p{};
        int64_t n_tiles = 0, rounds = 1, resident = 1;
        auto prepare = [&](const TileShape &t, bool whole) {
            cur = t;
            const int per_cu = precision == RAYSH_FP64 ? raysh::shoot_fp64_blocks_per_cu(t)
                                                       : raysh::shoot_fp32_blocks_per_cu(t);
            resident = (int64_t)per_cu * std::max(ctx->n_cu, 1);
            const raysh_rays s = shape_sample(*rays, t, ctx->n_stars, resident, n_tiles, rounds);
            p = ShootParams{};
            fill_shoot_params(p, ctx, whole ? rays : &s, pix);
            p.counts = scratch;
        };
        auto launch = [&](const TileShape &t) {
            return precision == RAYSH_FP64 ? raysh::launch_shoot_fp64(p, t, ctx->stream)
                                           : raysh::launch_shoot_fp32(p, t, ctx->stream);
        };
        std::vector<Timed> ranked;
        int code = time_shapes(
            precision, ctx->stream,
            [&](const TileShape &t) {
                if (std::memcmp(&t, &cur, sizeof t) != 0) prepare(t, false);
                return launch(t);
            },
            [&](const TileShape &t, double ms) {
                prepare(t, false);
                return ms / (double)rounds * (double)ceil_div(n_tiles, resident);
            },
            ranked);
        if (code == RAYSH_OK) {
            best = ranked[0].shape;
            best_ms = ranked[0].cost;
        }
        // The finalists (predictions within kFinalSpread of the best, at most
        // kFinalists) are timed on the whole block when it is short enough:
        // the per-round prediction cannot see everything a long launch does
        // (the clock it settles at, the last round's fill).
        if (code == RAYSH_OK && best_ms <= kFinalMaxMs) {
            hipEvent_t a, b;
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            double best_whole = -1;
            for (size_t i = 0; i < ranked.size() && (int)i < kFinalists && code == RAYSH_OK; ++i) {
                if (ranked[i].cost > best_ms * (1.0 + kFinalSpread)) break;
                prepare(ranked[i].shape, true);
                float fastest = 0;
                for (int rep = 0; rep < 2 && code == RAYSH_OK; ++rep) {
                    float ms = 0;
                    hipError_t e = hipEventRecord(a, ctx->stream);
                    if (e == hipSuccess) e = launch(ranked[i].shape);
                    if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                    if (e != hipSuccess) code = hip_error(e, "raysh_autotune");
                    if (rep == 0 || ms < fastest) fastest = ms;
                }
                if (code == RAYSH_OK && (best_whole < 0 || fastest < best_whole)) {
                    best_whole = fastest;
                    best = ranked[i].shape;
                }
            }
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (best_whole > 0) best_ms = best_whole;
        }
        (void)hipFree(scratch);
        if (code != RAYSH_OK) return code;
        if (cache_path) cache_store(cache_path, key, best, best_ms);
    }
    ctx->shape[precision] = best;
    report(best, cx, cy, share, star_tile);
    return set_ok();
}

extern "C" int raysh_autotune_batch(raysh_ctx *const *sets, int n_sets, const raysh_rays *rays,
                                    const raysh_pixels *pix, int precision, const char *cache_path, int *cx,
                                    int *cy, int *share, int *star_tile) {
    if (!sets || !rays || !pix) return set_error(RAYSH_EINVAL, "raysh_autotune_batch: NULL array");
    if (n_sets < 1) return set_error(RAYSH_EINVAL, "raysh_autotune_batch: n_sets < 1");
    if (int r = validate_tiled_precision(precision)) return r;
    int64_t total_stars = 0;
    for (int s = 0; s < n_sets; ++s) {
        if (!sets[s]) return set_error(RAYSH_EINVAL, "raysh_autotune_batch: set %d has no context", s);
        if (sets[s]->device != sets[0]->device)
            return set_error(RAYSH_EINVAL, "raysh_autotune_batch: contexts on different devices");
        if (int r = validate_rays(&rays[s])) return r;
        if (int r = validate_pixels(&pix[s])) return r;
        total_stars += sets[s]->n_stars;
    }
    raysh_ctx *lead = sets[0];
    DeviceGuard g(lead->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", lead->device);

    Key key;
    if (int r = make_key(lead->device, precision, "batch", total_stars / n_sets, key)) return r;
    if (!cache_path) cache_path = std::getenv("RAYSH_AUTOTUNE_CACHE");

    TileShape best{};
    double best_ms = -1;
    const bool cached = cache_path && cache_lookup(cache_path, key, best) && supported(precision, best);
    if (!cached) {
        // a sample batch: the central block of every set's rays, about an
        // equal share of kSampleWork each, its sides whole multiples of 128
        // rays (so that no compiled tile is ragged in it), at most the block
        std::vector<raysh_rays> sample(rays, rays + n_sets);
        for (int s = 0; s < n_sets; ++s) {
            const double want = kSampleWork / n_sets / (double)std::max<int64_t>(sets[s]->n_stars, 1);
            const int64_t side = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt(want) / 128.0)) * 128;
            raysh_rays &b = sample[s];
            b.nx = std::min<int64_t>(rays[s].nx, side);
            b.ny = std::min<int64_t>(rays[s].ny, side);
            b.i0 = rays[s].i0 + (rays[s].nx - b.nx) / 2;
            b.j0 = rays[s].j0 + (rays[s].ny - b.ny) / 2;
        }
        std::vector<int32_t *> maps(n_sets, nullptr);
        int code = RAYSH_OK;
        for (int s = 0; s < n_sets && code == RAYSH_OK; ++s) {
            if (hipMalloc(&maps[s], (size_t)pix[s].nx * (size_t)pix[s].ny * 4) != hipSuccess) {
                (void)hipGetLastError();
                maps[s] = nullptr;
                code = set_error(RAYSH_ENOMEM, "raysh_autotune_batch: scratch maps");
            }
        }
        std::vector<TileShape> old(n_sets);
        for (int s = 0; s < n_sets; ++s) old[s] = sets[s]->shape[precision];
        if (code == RAYSH_OK) {
            int inner = RAYSH_OK;
            std::vector<Timed> ranked;
            code = time_shapes(
                precision, lead->stream,
                [&](const TileShape &t) {
                    for (int s = 0; s < n_sets; ++s) sets[s]->shape[precision] = t;
                    inner = raysh_map_batch(sets, n_sets, sample.data(), pix, precision, maps.data());
                    return inner == RAYSH_OK ? hipSuccess : hipErrorLaunchFailure;
                },
                [](const TileShape &, double ms) { return ms; }, ranked);
            if (inner != RAYSH_OK) code = inner;   // keep the batch's own error
            if (code == RAYSH_OK) {
                best = ranked[0].shape;
                best_ms = ranked[0].cost;
            }
        }
        (void)hipStreamSynchronize(lead->stream);   // the scratch maps are still written
        for (int32_t *m : maps)
            if (m) (void)hipFree(m);
        if (code != RAYSH_OK) {
            for (int s = 0; s < n_sets; ++s) sets[s]->shape[precision] = old[s];
            return code;
        }
        if (cache_path) cache_store(cache_path, key, best, best_ms);
    }
    for (int s = 0; s < n_sets; ++s) sets[s]->shape[precision] = best;
    report(best, cx, cy, share, star_tile);
    return set_ok();
}
