// Host side of the raysh C ABI: argument validation, contexts, star upload
// and kernel dispatch.  The operation itself is Eq. (1)-(3) and Algorithm 1
// of arXiv:1703.09707 (see include/raysh.h for the conventions).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "raysh_ctx.h"

using raysh::ShootParams;
using raysh::Star;
using raysh::TileShape;


namespace {

thread_local char g_err[512] = "";
constexpr int64_t kMaxRays = std::numeric_limits<int32_t>::max();
constexpr int64_t kMaxIndex = int64_t(1) << 53;

constexpr size_t kMaxSplitBytes = size_t(2) << 30;   // automatic split-K workspace cap
constexpr int64_t kCellAutoStars = 65536;             // star cells by default from this many stars on
constexpr int kMinStarsPerPart = 64;

// Parts of the FP64 star sum for a call (1 = one pass): `want` >= 1 as
// given, 0 automatic with a workspace of at most cap_bytes.
int split_parts(const raysh_ctx *c, const ShootParams &p, int want, size_t cap_bytes) {
    if (want >= 1) return want;   // as set (1 = one pass)
    // automatic: enough (tile, part) workgroups to fill the GPU several times
    if (c->n_stars < 2 * kMinStarsPerPart) return 1;
    const int64_t n_rays = p.nx * p.ny;
    const TileShape &t = c->shape[0];
    const int64_t tiles = ((p.nx + raysh::tile_width(t) - 1) / raysh::tile_width(t)) *
                          ((p.ny + raysh::tile_height(t) - 1) / raysh::tile_height(t));
    const int64_t want_blocks = (int64_t)std::max(c->n_cu, 1) * 8;   // several waves of workgroups
    int64_t parts = (want_blocks + tiles - 1) / tiles;
    parts = std::min<int64_t>(parts, c->n_stars / kMinStarsPerPart);
    parts = std::min<int64_t>(parts, (int64_t)(cap_bytes / (16 * (size_t)n_rays)));
    return (int)std::max<int64_t>(parts, 1);
}

// Allocation-free FP64 map: the split star sum's partial sums go to this
// file-scope device array instead of a context workspace.  Each device
// holds its own copy until the process ends; its address is resolved once
// per device (bind_scratch, from raysh_init) and only that address is used
// on the host side.  Calls that overlap on one device share it and race.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// With `device` current: the device address of `scratch` on it, resolved
// on the first call for the device.
hipError_t bind_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

int launch(raysh_ctx *c, const ShootParams &p, int precision, const char *what) {
    hipError_t e;
    if (precision == RAYSH_FP64) {
        const int parts = split_parts(c, p, c->star_parts, kMaxSplitBytes);
        if (parts > 1) {
            const size_t need = (size_t)parts * (size_t)(p.nx * p.ny) * sizeof(double2);
            if (need > c->partial_bytes) {
                e = hipStreamSynchronize(c->stream);   // the old workspace may still be read
                if (e != hipSuccess) return hip_error(e, what);
                if (c->d_partial) (void)hipFree(c->d_partial);
                c->d_partial = nullptr;
                c->partial_bytes = 0;
                e = hipMalloc(&c->d_partial, need);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    c->d_partial = nullptr;
                    return set_error(RAYSH_ENOMEM, "%s: split-K workspace of %zu bytes", what, need);
                }
                c->partial_bytes = need;
            }
            e = raysh::launch_split_fp64(p, c->shape[0], parts, c->d_partial, c->stream);
        } else {
            e = raysh::launch_shoot_fp64(p, c->shape[0], c->stream);
        }
    } else if (precision == RAYSH_FP32_BULK) {
        e = raysh::launch_shoot_fp32(p, c->shape[1], c->stream);
    } else {
        raysh::StarCells cells{};   // ncx = 0: the block pass visits every star
        const bool want = c->expansion_cells == RAYSH_CELLS_ALWAYS ||
                          (c->expansion_cells == RAYSH_CELLS_AUTO && c->n_stars >= kCellAutoStars);
        if (want) {
            if (!c->cells_built) {
                e = raysh::build_star_cells(c->d_stars, c->n_stars, c->stream, c->cells);
                if (e == hipErrorOutOfMemory) {
                    (void)hipGetLastError();
                    return set_error(RAYSH_ENOMEM, "%s: star cells of %lld stars", what, (long long)c->n_stars);
                }
                if (e != hipSuccess) return hip_error(e, what);
                c->cells_built = true;
            }
            cells = c->cells.view;
        }
        const int block =
            c->expansion_block ? c->expansion_block : raysh::expansion_block(p.nx, p.ny, c->n_stars, c->n_cu);
        const size_t need = raysh::expansion_workspace_bytes(p.nx, p.ny, block);
        if (need > c->far_bytes) {
            e = hipStreamSynchronize(c->stream);   // the old workspace may still be read
            if (e != hipSuccess) return hip_error(e, what);
            if (c->d_far) (void)hipFree(c->d_far);
            c->d_far = nullptr;
            c->far_bytes = 0;
            e = hipMalloc(&c->d_far, need);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                c->d_far = nullptr;
                return set_error(RAYSH_ENOMEM, "%s: expansion workspace of %zu bytes", what, need);
            }
            c->far_bytes = need;
        }
        e = raysh::launch_shoot_expansion(p, cells, c->theta_open, block, c->d_far, c->stream);
    }
    if (e != hipSuccess) return hip_error(e, what);
    return RAYSH_OK;
}

// Star records go to the device through two pinned staging buffers of
// kUploadChunk records, packed on the host while the other one is copied,
// so the host holds 2 x 16 MiB at any N* instead of a second copy of the
// star field.  The buffers stay with the context (raysh_set_lens uploads
// through them again).  Synchronous: returns when every record is on the
// device.
constexpr size_t kUploadChunk = size_t(1) << 19;

hipError_t upload_stars(raysh_ctx *c, const raysh_lens *lens, size_t total) {
    const size_t per = std::min(kUploadChunk, total);
    const int n_buf = total > per ? 2 : 1;
    hipError_t e = hipSuccess;
    if (c->stage_records < per) {
        for (int b = 0; b < 2; ++b) {
            if (c->h_stage[b]) (void)hipHostFree(c->h_stage[b]);
            c->h_stage[b] = nullptr;
        }
        c->stage_records = per;
    }
    for (int b = 0; b < n_buf && e == hipSuccess; ++b)
        if (!c->h_stage[b]) e = hipHostMalloc((void **)&c->h_stage[b], c->stage_records * sizeof(Star),
                                              hipHostMallocDefault);
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    for (int b = 0; b < n_buf && e == hipSuccess; ++b) e = hipEventCreateWithFlags(&done[b], hipEventDisableTiming);
    for (size_t off = 0, b = 0; off < total && e == hipSuccess; off += per, b = (b + 1) % n_buf) {
        const size_t cnt = std::min(per, total - off);
        if (pending[b]) e = hipEventSynchronize(done[b]);   // the buffer's last copy has finished
        if (e != hipSuccess) break;
        Star *stage = c->h_stage[b];
        for (size_t k = 0; k < cnt; ++k) {
            const size_t i = off + k;
            stage[k] = (int64_t)i < lens->n_stars ? Star{lens->x[i], lens->y[i], lens->m[i], 0.0}
                                                   : Star{0.0, 0.0, 0.0, 0.0};
        }
        e = hipMemcpyAsync(c->d_stars + off, stage, cnt * sizeof(Star), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipEventRecord(done[b], c->stream);
        pending[b] = e == hipSuccess;
    }
    const hipError_t s = hipStreamSynchronize(c->stream);   // the staging buffers are free again
    if (e == hipSuccess) e = s;
    for (int b = 0; b < 2; ++b)
        if (done[b]) (void)hipEventDestroy(done[b]);
    return e;
}

// The checks raysh_init and raysh_set_lens make on a lens.
int validate_lens(const raysh_lens *lens) {
    if (!lens) return set_error(RAYSH_EINVAL, "lens is NULL");
    if (!std::isfinite(lens->kappa_c) || !std::isfinite(lens->gamma1) || !std::isfinite(lens->gamma2))
        return set_error(RAYSH_EINVAL, "kappa_c and gamma must be finite");
    if (lens->n_stars < 0) return set_error(RAYSH_EINVAL, "n_stars < 0");
    if (lens->n_stars > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "n_stars > 2^31-1");
    const int64_t n = lens->n_stars;
    if (n > 0 && (!lens->x || !lens->y || !lens->m)) return set_error(RAYSH_EINVAL, "star array is NULL");
    for (int64_t k = 0; k < n; ++k) {
        if (!std::isfinite(lens->x[k]) || !std::isfinite(lens->y[k]))
            return set_error(RAYSH_EINVAL, "star %lld position is not finite", (long long)k);
        if (!std::isfinite(lens->m[k]) || lens->m[k] < 0)
            return set_error(RAYSH_EINVAL, "star %lld mass is negative or not finite", (long long)k);
    }
    return RAYSH_OK;
}

void set_macro(raysh_ctx *c, const raysh_lens *lens) {
    c->kappa_c = lens->kappa_c;
    c->gamma1 = lens->gamma1;
    c->gamma2 = lens->gamma2;
    c->k11 = lens->kappa_c + lens->gamma1;
    c->k12 = lens->gamma2;
    c->k22 = lens->kappa_c - lens->gamma1;
}

}  // namespace

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int set_ok() {
    g_err[0] = '\0';
    return RAYSH_OK;
}

int hip_error(hipError_t e, const char *what) {
    return set_error(RAYSH_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int validate_rays(const raysh_rays *r) {
    if (!r) return set_error(RAYSH_EINVAL, "rays is NULL");
    if (!std::isfinite(r->x0) || !std::isfinite(r->y0))
        return set_error(RAYSH_EINVAL, "ray lattice origin is not finite");
    if (!(std::isfinite(r->dx) && r->dx > 0) || !(std::isfinite(r->dy) && r->dy > 0))
        return set_error(RAYSH_EINVAL, "ray spacing must be finite and > 0");
    if (r->nx < 0 || r->ny < 0) return set_error(RAYSH_EINVAL, "ray counts must be >= 0");
    if (r->i0 < 0 || r->j0 < 0) return set_error(RAYSH_EINVAL, "ray block offsets must be >= 0");
    if (r->i0 > kMaxIndex - r->nx || r->j0 > kMaxIndex - r->ny)
        return set_error(RAYSH_EOVERFLOW, "ray lattice index beyond 2^53");
    if (r->nx > 0 && r->ny > kMaxRays / r->nx)
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 rays in one call");
    const double ex = r->x0 + ((double)(r->i0 + r->nx) + 0.5) * r->dx;
    const double ey = r->y0 + ((double)(r->j0 + r->ny) + 0.5) * r->dy;
    if (!std::isfinite(ex) || !std::isfinite(ey))
        return set_error(RAYSH_EINVAL, "image angles of the lattice are not finite");
    return RAYSH_OK;
}

int validate_pixels(const raysh_pixels *p) {
    if (!p) return set_error(RAYSH_EINVAL, "pixels is NULL");
    if (!std::isfinite(p->x0) || !std::isfinite(p->y0))
        return set_error(RAYSH_EINVAL, "source window origin is not finite");
    if (!(std::isfinite(p->px) && p->px > 0) || !(std::isfinite(p->py) && p->py > 0))
        return set_error(RAYSH_EINVAL, "pixel size must be finite and > 0");
    if (p->nx <= 0 || p->ny <= 0) return set_error(RAYSH_EINVAL, "pixel counts must be > 0");
    if ((int64_t)p->ny > kMaxRays / (int64_t)p->nx)
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 pixels");
    if (!std::isfinite(p->x0 + p->nx * p->px) || !std::isfinite(p->y0 + p->ny * p->py))
        return set_error(RAYSH_EINVAL, "source window is not finite");
    return RAYSH_OK;
}

int validate_precision(int precision) {
    if (precision != RAYSH_FP64 && precision != RAYSH_FP32_BULK && precision != RAYSH_FP64_EXPANSION)
        return set_error(RAYSH_EINVAL, "unknown precision %d", precision);
    return RAYSH_OK;
}

int validate_tiled_precision(int precision) {
    if (precision != RAYSH_FP64 && precision != RAYSH_FP32_BULK)
        return set_error(RAYSH_EINVAL,
                         "precision %d: launch shapes, batches and tuning apply to RAYSH_FP64 and RAYSH_FP32_BULK",
                         precision);
    return RAYSH_OK;
}

int validate_device_ptr(const void *ptr, size_t bytes, int device, const char *name) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "%s is not device memory", name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return set_error(RAYSH_EINVAL, "%s is not device memory", name);
    if (attr.device != device)
        return set_error(RAYSH_EINVAL, "%s is on device %d, the context on %d", name, attr.device,
                         device);
    void *base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void *>(ptr));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "%s: cannot query its allocation", name);
    }
    const size_t off = (size_t)((const char *)ptr - (const char *)base);
    if (off > size || size - off < bytes)
        return set_error(RAYSH_EINVAL, "%s holds %zu bytes, %zu needed", name, size - off, bytes);
    return RAYSH_OK;
}

void fill_shoot_params(ShootParams &p, const raysh_ctx *c, const raysh_rays *r,
                       const raysh_pixels *w) {
    p.k11 = c->k11;
    p.k12 = c->k12;
    p.k22 = c->k22;
    p.stars = c->d_stars;
    p.n_stars = (int32_t)c->n_stars;
    p.x0 = r->x0;
    p.y0 = r->y0;
    p.dx = r->dx;
    p.dy = r->dy;
    p.nx = r->nx;
    p.ny = r->ny;
    p.i0 = r->i0;
    p.j0 = r->j0;
    p.X0 = w->x0;
    p.Y0 = w->y0;
    p.Px = w->px;
    p.Py = w->py;
    p.NX = w->nx;
    p.NY = w->ny;
}

extern "C" {

const char *raysh_last_error(void) { return g_err; }

int raysh_init(raysh_ctx **out, const raysh_lens *lens, int device, void *hip_stream) {
    if (!out) return set_error(RAYSH_EINVAL, "out is NULL");
    if (int r = validate_lens(lens)) return r;
    const int64_t n = lens->n_stars;
    if (device < 0) return set_error(RAYSH_EINVAL, "device < 0");
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
    if (device >= n_dev) return set_error(RAYSH_EINVAL, "device %d of %d", device, n_dev);

    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    void *static_scratch = nullptr;
    e = bind_scratch(device, &static_scratch);
    if (e != hipSuccess) return hip_error(e, "raysh_init: static scratch of raysh_map_split_noalloc");
    raysh_ctx *c = new raysh_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->n_stars = n;
    set_macro(c, lens);
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        (void)hipGetLastError();
        c->n_cu = 1;
    }

    const size_t total = (size_t)(n > 0 ? n : 1);   // one zero record when there are no stars
    e = hipMalloc(&c->d_stars, total * sizeof(Star));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return set_error(RAYSH_ENOMEM, "device allocation of %zu stars failed", total);
    }
    c->star_capacity = (int64_t)total;
    e = hipMalloc(&c->d_counter, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc(&c->h_counter, sizeof(unsigned long long), hipHostMallocDefault);
    if (e == hipSuccess) e = upload_stars(c, lens, total);
    if (e != hipSuccess) {
        int code = hip_error(e, "raysh_init");
        raysh_free(c);
        return code;
    }
    *out = c;
    return set_ok();
}

int raysh_set_lens(raysh_ctx *ctx, const raysh_lens *lens) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (int r = validate_lens(lens)) return r;
    const int64_t n = lens->n_stars;
    const size_t total = (size_t)(n > 0 ? n : 1);   // one zero record when there are no stars
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    // work enqueued before this call may read the old stars: on the
    // context's stream, and in a batch led by another context, on its
    // stream; so the whole device drains first
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "raysh_set_lens");
    if ((int64_t)total > ctx->star_capacity) {
        // grow by half again at least, so that a run of growing fields reallocates rarely
        const size_t cap = std::max(total, (size_t)ctx->star_capacity + (size_t)ctx->star_capacity / 2);
        Star *grown = nullptr;
        e = hipMalloc(&grown, cap * sizeof(Star));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(RAYSH_ENOMEM, "raysh_set_lens: device allocation of %zu stars failed", cap);
        }
        (void)hipFree(ctx->d_stars);
        ctx->d_stars = grown;
        ctx->star_capacity = (int64_t)cap;
    }
    raysh_forget_batches(ctx);             // captured batches hold the old star count
    raysh::free_star_cells(ctx->cells);    // built again, from the new stars, when used
    ctx->cells_built = false;
    ctx->n_stars = n;
    set_macro(ctx, lens);
    e = upload_stars(ctx, lens, total);
    if (e != hipSuccess) return hip_error(e, "raysh_set_lens");
    return set_ok();
}

int raysh_set_expansion(raysh_ctx *ctx, double theta_open) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (!(theta_open > 0.0 && theta_open <= 0.3))
        return set_error(RAYSH_EINVAL, "theta_open must lie in (0, 0.3]");
    ctx->theta_open = theta_open;
    return set_ok();
}

int raysh_set_expansion_cells(raysh_ctx *ctx, int mode) {
    if (!ctx) return set_error(RAYSH_EINVAL, "raysh_set_expansion_cells: NULL context");
    if (mode != RAYSH_CELLS_AUTO && mode != RAYSH_CELLS_ALWAYS && mode != RAYSH_CELLS_NEVER)
        return set_error(RAYSH_EINVAL, "expansion cells mode must be RAYSH_CELLS_AUTO, _ALWAYS or _NEVER");
    ctx->expansion_cells = mode;
    return set_ok();
}

int raysh_set_expansion_block(raysh_ctx *ctx, int block) {
    if (!ctx) return set_error(RAYSH_EINVAL, "raysh_set_expansion_block: NULL context");
    if (block != 0 && block != 1 && block != 2 && block != 4)
        return set_error(RAYSH_EINVAL, "expansion block must be 0 (automatic), 1, 2 or 4");
    ctx->expansion_block = block;
    return set_ok();
}

int raysh_expansion_order(void) { return raysh::expansion_order(); }

int raysh_set_star_split(raysh_ctx *ctx, int parts) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (parts < 0 || parts > 65536) return set_error(RAYSH_EINVAL, "star split %d outside [0, 65536]", parts);
    ctx->star_parts = parts;
    return set_ok();
}

int raysh_set_stream(raysh_ctx *ctx, void *hip_stream) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return set_ok();
}

int64_t raysh_n_stars(const raysh_ctx *ctx) { return ctx ? ctx->n_stars : 0; }

int raysh_set_tile(raysh_ctx *ctx, int precision, int cx, int cy, int share, int star_tile) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (int r = validate_tiled_precision(precision)) return r;
    if (precision == RAYSH_FP32_BULK && share != 0)
        return set_error(RAYSH_EINVAL, "share does not apply to RAYSH_FP32_BULK and must be 0");
    if (precision == RAYSH_FP64 && star_tile == 0) star_tile = share < 4 ? share : 4;   // stars per group
    TileShape t{cx, cy, share, star_tile};
    const bool supported = precision == RAYSH_FP64 ? raysh::fp64_shape_supported(t)
                                                   : raysh::fp32_shape_supported(t);
    if (!supported)
        return set_error(RAYSH_EINVAL, "tile shape (%d, %d, %d, %d) is not built for precision %d", cx, cy,
                    share, star_tile, precision);
    ctx->shape[precision] = t;
    return set_ok();
}

int raysh_list_tiles(int precision, int32_t *shapes, int cap) {
    if (validate_tiled_precision(precision) != RAYSH_OK || cap < 0 || (cap > 0 && !shapes)) {
        set_error(RAYSH_EINVAL, "raysh_list_tiles: bad precision, cap or NULL shapes");
        return -RAYSH_EINVAL;
    }
    TileShape t[64];
    const int n = precision == RAYSH_FP64 ? raysh::fp64_shape_list(t, 64) : raysh::fp32_shape_list(t, 64);
    for (int i = 0; i < n && i < cap && i < 64; ++i) {
        shapes[4 * i + 0] = t[i].cx;
        shapes[4 * i + 1] = t[i].cy;
        shapes[4 * i + 2] = t[i].share;
        shapes[4 * i + 3] = t[i].star_tile;
    }
    set_ok();
    return n;
}

int raysh_get_tile(const raysh_ctx *ctx, int precision, int *cx, int *cy, int *share, int *star_tile) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (int r = validate_tiled_precision(precision)) return r;
    const TileShape &t = ctx->shape[precision];
    if (cx) *cx = t.cx;
    if (cy) *cy = t.cy;
    if (share) *share = t.share;
    if (star_tile) *star_tile = t.star_tile;
    return set_ok();
}

int raysh_shoot(raysh_ctx *ctx, const raysh_rays *rays, int precision, double *beta_x,
                double *beta_y, const raysh_pixels *pix, int32_t *bin) {
    if (int r = validate_rays(rays)) return r;
    if (int r = validate_precision(precision)) return r;
    if (bin && !pix) return set_error(RAYSH_EINVAL, "bin requested without a source window");
    if (pix)
        if (int r = validate_pixels(pix)) return r;
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    const int64_t n = rays->nx * rays->ny;
    if (n == 0) return set_ok();
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    if (beta_x)
        if (int r = validate_device_ptr(beta_x, (size_t)n * 8, ctx->device, "beta_x")) return r;
    if (beta_y)
        if (int r = validate_device_ptr(beta_y, (size_t)n * 8, ctx->device, "beta_y")) return r;
    if (bin)
        if (int r = validate_device_ptr(bin, (size_t)n * 4, ctx->device, "bin")) return r;
    if (!beta_x && !beta_y && !bin) return set_ok();

    static const raysh_pixels unit = {0.0, 0.0, 1.0, 1.0, 1, 1};
    ShootParams p{};
    fill_shoot_params(p, ctx, rays, pix ? pix : &unit);
    p.beta_x = beta_x;
    p.beta_y = beta_y;
    p.bin = bin;
    if (int r = launch(ctx, p, precision, "raysh_shoot")) return r;
    return set_ok();
}

int raysh_map(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix, int precision,
              int32_t *counts, uint64_t *n_binned) {
    if (int r = validate_rays(rays)) return r;
    if (int r = validate_pixels(pix)) return r;
    if (int r = validate_precision(precision)) return r;
    if (!counts) return set_error(RAYSH_EINVAL, "counts is NULL");
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    const size_t map_bytes = (size_t)pix->nx * (size_t)pix->ny * 4;
    if (int r = validate_device_ptr(counts, map_bytes, ctx->device, "counts")) return r;
    const int64_t n = rays->nx * rays->ny;
    if (n == 0) {
        if (n_binned) *n_binned = 0;
        return set_ok();
    }
    ShootParams p{};
    fill_shoot_params(p, ctx, rays, pix);
    p.counts = counts;
    hipError_t e = hipSuccess;
    if (n_binned) {
        p.n_binned = ctx->d_counter;
        e = raysh::launch_zero_u64(ctx->d_counter, 1, ctx->stream);
        if (e != hipSuccess) return hip_error(e, "raysh_map counter reset");
    }
    if (int r = launch(ctx, p, precision, "raysh_map")) return r;
    if (n_binned) {
        e = hipMemcpyAsync(ctx->h_counter, ctx->d_counter, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_error(e, "raysh_map");
        *n_binned = *ctx->h_counter;
    }
    return set_ok();
}

int raysh_map_split_noalloc(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix, int parts,
                            int32_t *counts) {
    if (int r = validate_rays(rays)) return r;
    if (int r = validate_pixels(pix)) return r;
    if (!counts) return set_error(RAYSH_EINVAL, "counts is NULL");
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    if (parts < 0 || parts > 65536) return set_error(RAYSH_EINVAL, "star split %d outside [0, 65536]", parts);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    const size_t map_bytes = (size_t)pix->nx * (size_t)pix->ny * 4;
    if (int r = validate_device_ptr(counts, map_bytes, ctx->device, "counts")) return r;
    const int64_t n = rays->nx * rays->ny;
    if (n == 0) return set_ok();
    ShootParams p{};
    fill_shoot_params(p, ctx, rays, pix);
    p.counts = counts;
    const int use = split_parts(ctx, p, parts, kStaticScratchBytes);
    const size_t need = (size_t)use * (size_t)n * sizeof(double2);
    if (use > 1 && need > kStaticScratchBytes)
        return set_error(RAYSH_EOVERFLOW,
                         "raysh_map_split_noalloc: %d parts of %lld rays need %zu bytes of partial sums, "
                         "beyond its static scratch of %zu bytes",
                         use, (long long)n, need, kStaticScratchBytes);
    void *ptr = nullptr;
    hipError_t e = bind_scratch(ctx->device, &ptr);   // resolved by raysh_init; no allocation here
    if (e != hipSuccess) return hip_error(e, "raysh_map_split_noalloc");
    e = use > 1 ? raysh::launch_split_fp64(p, ctx->shape[0], use, static_cast<double2 *>(ptr), ctx->stream)
                : raysh::launch_shoot_fp64(p, ctx->shape[0], ctx->stream);
    if (e != hipSuccess) return hip_error(e, "raysh_map_split_noalloc");
    return set_ok();
}

int raysh_sync(raysh_ctx *ctx) {
    if (!ctx) return set_error(RAYSH_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_error(e, "raysh_sync");
    return set_ok();
}

int raysh_free(raysh_ctx *ctx) {
    if (!ctx) return set_ok();
    raysh_forget_batches(ctx);
    int code = RAYSH_OK;
    {
        DeviceGuard g(ctx->device);
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) code = RAYSH_EDEVICE;
        if (ctx->d_stars) (void)hipFree(ctx->d_stars);
        if (ctx->d_counter) (void)hipFree(ctx->d_counter);
        if (ctx->d_partial) (void)hipFree(ctx->d_partial);
        if (ctx->d_far) (void)hipFree(ctx->d_far);
        if (ctx->h_counter) (void)hipHostFree(ctx->h_counter);
        for (int b = 0; b < 2; ++b)
            if (ctx->h_stage[b]) (void)hipHostFree(ctx->h_stage[b]);
        raysh::free_star_cells(ctx->cells);
    }
    delete ctx;
    if (code != RAYSH_OK) return set_error(code, "raysh_free: pending device error");
    return set_ok();
}

}  // extern "C"
