// Launch-shape autotuner: times every compiled tile shape of one precision
// on a sample of the caller's ray block and keeps the fastest in the
// context.  Choices are cached in a plain text file, one line per key:
//   <arch> <cus> <precision> <log2 stars bucket> <cx> <cy> <share> <star_tile> <ms>
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
    char arch[128];
    int cus, prec, bucket, cx, cy, share, st;
    double ms;
    bool found = false;
    while (std::fscanf(f, "%127s %d %d %d %d %d %d %d %lf", arch, &cus, &prec, &bucket, &cx, &cy, &share,
                       &st, &ms) == 9) {
        if (k.arch == arch && k.cus == cus && k.precision == prec && k.bucket == bucket) {
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
    std::fprintf(f, "%s %d %d %d %d %d %d %d %.4f\n", k.arch.c_str(), k.cus, k.precision, k.bucket, t.cx,
                 t.cy, t.share, t.star_tile, ms);
    std::fclose(f);
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

    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) return hip_error(e, "raysh_autotune");
    Key key;
    key.arch = prop.gcnArchName;
    for (char &c : key.arch)
        if (c == ' ') c = '_';
    key.cus = prop.multiProcessorCount;
    key.precision = precision;
    key.bucket = star_bucket(ctx->n_stars);
    if (!cache_path) cache_path = std::getenv("RAYSH_AUTOTUNE_CACHE");

    TileShape best{};
    double best_ms = -1;
    const bool cached = cache_path && cache_lookup(cache_path, key, best) &&
                        (precision == RAYSH_FP64 ? raysh::fp64_shape_supported(best)
                                                 : raysh::fp32_shape_supported(best));
    if (!cached) {
        // central sample of about 2e10 / N* rays (at least 256^2, at most the block)
        const double want = std::max(65536.0, 2e10 / (double)std::max<int64_t>(ctx->n_stars, 1));
        int64_t side = (int64_t)std::sqrt(want);
        raysh_rays s = *rays;
        s.nx = std::min<int64_t>(rays->nx, side);
        s.ny = std::min<int64_t>(rays->ny, side);
        s.i0 = rays->i0 + (rays->nx - s.nx) / 2;
        s.j0 = rays->j0 + (rays->ny - s.ny) / 2;
        if (s.nx == 0 || s.ny == 0) return set_error(RAYSH_EINVAL, "raysh_autotune: empty ray block");

        int32_t *scratch = nullptr;
        const size_t map_bytes = (size_t)pix->nx * (size_t)pix->ny * 4;
        e = hipMalloc(&scratch, map_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(RAYSH_ENOMEM, "raysh_autotune: scratch map");
        }
        hipEvent_t t0, t1;
        (void)hipEventCreate(&t0);
        (void)hipEventCreate(&t1);
        ShootParams p{};
        fill_shoot_params(p, ctx, &s, pix);
        p.counts = scratch;
        TileShape shapes[32];
        int n_shapes = precision == RAYSH_FP64 ? raysh::fp64_shape_list(shapes, 32)
                                               : raysh::fp32_shape_list(shapes, 32);
        n_shapes = std::min(n_shapes, 32);
        int code = RAYSH_OK;
        for (int i = 0; i < n_shapes && code == RAYSH_OK; ++i) {
            const TileShape &t = shapes[i];
            auto run = [&]() {
                return precision == RAYSH_FP64 ? raysh::launch_shoot_fp64(p, t, ctx->stream)
                                               : raysh::launch_shoot_fp32(p, t, ctx->stream);
            };
            e = run();   // warm-up
            if (e == hipSuccess) e = hipEventRecord(t0, ctx->stream);
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = run();
            if (e == hipSuccess) e = hipEventRecord(t1, ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e != hipSuccess) {
                code = hip_error(e, "raysh_autotune");
                break;
            }
            if (best_ms < 0 || ms / 3 < best_ms) {
                best_ms = ms / 3;
                best = t;
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        (void)hipFree(scratch);
        if (code != RAYSH_OK) return code;
        if (cache_path) cache_store(cache_path, key, best, best_ms);
    }
    ctx->shape[precision] = best;
    if (cx) *cx = best.cx;
    if (cy) *cy = best.cy;
    if (share) *share = best.share;
    if (star_tile) *star_tile = best.star_tile;
    return set_ok();
}
