// Simulated light curves: the map seen by a source of finite size, sampled
// along straight tracks.
//
// A magnification map together with a model of the source's size and
// brightness profile yields simulated microlensing light curves
// (arXiv:1703.09707, Sec. 1).  The paper fixes neither the profile nor the
// tracks; this library offers
//   * a circular Gaussian (the separable smoothing of smooth.h), and
//   * a uniform disk of radius R: the pixels at offsets (k, l) with
//     (k Px)^2 + (l Py)^2 <= R^2 (FP64, each square a product of its own),
//     averaged as (norm * S) / n with S the exact integer sum of their
//     counts and n their number;
// and straight tracks a -> b sampled at n evenly spaced points, computed in
// the source map's centre-index space (u_k = u_a + k du with
// u_a = (xa - x0) (1/px) - 0.5 and du = ((xb - xa) (1/px)) (1/(n - 1)),
// each reciprocal rounded once), interpolated bilinearly between the four
// surrounding pixel centres (NaN outside the hull of the centres).
//
// The light-curve kernel is a gather: each sample reads four map values and
// writes one.  Consecutive lanes take consecutive samples of one track, so
// a wave's reads fall on a few neighbouring rows of the map, which stays in
// L2 (a 1024^2 FP64 map is 8 MiB).  Its HBM traffic is the curves written
// plus the map read once.  The curves are written with non-temporal
// (streaming) stores: they are not read again by the kernel, and held in the
// caches they would take the room and the bandwidth the map's lines need.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "raysh_ctx.h"
#include "smooth.h"

namespace {

constexpr int kLcThreads = 256;

// The disk test, the same FP64 expression on the host and the device.
__host__ __device__ inline bool disk_in(int k, int l, double px, double py, double radius) {
#pragma clang fp contract(off)
    const double a = (double)k * px;
    const double b = (double)l * py;
    return a * a + b * b <= radius * radius;
}

// Half-widths of the disk along row 0 and column 0.  The caller has checked
// that radius / px < nx and radius / py < ny, which bounds both scans.
void disk_radii(double radius, double px, double py, int *rx, int *ry) {
    int a = 0;
    while (disk_in(a + 1, 0, px, py, radius)) ++a;
    int b = 0;
    while (disk_in(0, b + 1, px, py, radius)) ++b;
    *rx = a;
    *ry = b;
}

// half[l + ry] = largest k >= 0 with disk_in(k, l), for |l| <= ry; then
// n_taps = sum over rows of (2 half + 1).  One workgroup.
__global__ __launch_bounds__(kLcThreads) void disk_rows_kernel(double radius, double px, double py, int rx,
                                                               int ry, int *half, long long *n_taps) {
    __shared__ long long part[kLcThreads];
    long long cnt = 0;
    for (int r = threadIdx.x; r <= 2 * ry; r += kLcThreads) {
        const int l = r - ry;
        int k = 0;
        while (k < rx && disk_in(k + 1, l, px, py, radius)) ++k;
        half[r] = k;
        cnt += 2 * k + 1;
    }
    part[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int i = 0; i < kLcThreads; ++i) t += part[i];
        *n_taps = t;
    }
}

// mu_s[j][i] = (norm * S) / n, S = sum of counts over the disk around
// pixel (i + rx, j + ry).
__global__ __launch_bounds__(kLcThreads) void disk_map_kernel(const int32_t *__restrict__ counts, int nx,
                                                              double norm, int rx, int ry,
                                                              const int *__restrict__ half,
                                                              const long long *__restrict__ n_taps, int wx,
                                                              int wy, double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * kLcThreads + threadIdx.x;
    if (idx >= (int64_t)wx * wy) return;
    const int j = (int)(idx / wx), i = (int)(idx % wx);
    long long s = 0;
    for (int r = 0; r <= 2 * ry; ++r) {
        const int h = half[r];
        const int32_t *row = counts + (int64_t)(j + r) * nx + (i + rx);
        for (int k = -h; k <= h; ++k) s += row[k];
    }
    out[idx] = (norm * (double)s) / (double)(*n_taps);
}

// kSpt samples per lane, kLcThreads apart: a block covers kSpt * kLcThreads
// consecutive (track, sample) pairs, and each of a lane's stores is part of
// one coalesced wave-wide store.  The block's first pair is found once, with
// a uniform 64-bit division; a lane's offset r < n + kSpt * kLcThreads from
// there splits into (track, sample) with a single-precision reciprocal,
// whose quotient is within one of the exact one (relative error below 2^-21
// on a quotient of at most kSpt * kLcThreads), and one correction step.
// Each sample sets up its track in centre-index space (u_a, du) with the
// host's reciprocals, so no lane divides.  The body has no branches: all
// loads of a lane are issued before the first wait, indices are clamped to
// a valid pixel before any conversion, and the value is selected at the end.
constexpr int kSpt = 4;

__global__ __launch_bounds__(kLcThreads) void light_curve_kernel(
    const double *__restrict__ mu, int nx, int ny, double x0, double y0, double ipx, double ipy,
    const double *__restrict__ xa, const double *__restrict__ ya, const double *__restrict__ xb,
    const double *__restrict__ yb, const int32_t *__restrict__ order, const double *__restrict__ sorted,
    int64_t n_tracks, int n_samples, float inv_nf, double inv_n1, double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t base = (int64_t)blockIdx.x * (kSpt * kLcThreads);
    const int64_t total = n_tracks * (int64_t)n_samples;
    const int64_t t0 = base / n_samples;
    const int r0 = (int)(base - t0 * n_samples) + (int)threadIdx.x;
    int64_t t[kSpt], tv[kSpt];   // track (row of out), and its visit index
    int k[kSpt];
    bool live[kSpt];
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        const int r = r0 + e * kLcThreads;   // < n_samples + kSpt * kLcThreads <= 2^24 + 1024
        int q = (int)((float)r * inv_nf);
        int kk = r - q * n_samples;
        if (kk < 0) {
            --q;
            kk += n_samples;
        } else if (kk >= n_samples) {
            ++q;
            kk -= n_samples;
        }
        live[e] = base + threadIdx.x + e * kLcThreads < total;
        int64_t tt = t0 + q;
        tv[e] = live[e] ? tt : 0;
        if (order && live[e]) {
            tt = order[tt];
            live[e] = tt >= 0 && tt < n_tracks;   // entries outside the tracks are skipped
        }
        t[e] = live[e] ? tt : 0;   // a lane with nothing to do reads track 0 and stores nothing
        k[e] = kk;
    }
    double ax[kSpt], ay[kSpt], bx[kSpt], by[kSpt];
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        if (sorted) {
            ax[e] = sorted[tv[e]];
            ay[e] = sorted[n_tracks + tv[e]];
            bx[e] = sorted[2 * n_tracks + tv[e]];
            by[e] = sorted[3 * n_tracks + tv[e]];
        } else {
            ax[e] = xa[t[e]];
            ay[e] = ya[t[e]];
            bx[e] = xb[t[e]];
            by[e] = yb[t[e]];
        }
    }
    double fx[kSpt], fy[kSpt], m00[kSpt], m01[kSpt], m10[kSpt], m11[kSpt];
    bool inside[kSpt];
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        const double ua = (ax[e] - x0) * ipx - 0.5;
        const double va = (ay[e] - y0) * ipy - 0.5;
        const double du = ((bx[e] - ax[e]) * ipx) * inv_n1;
        const double dv = ((by[e] - ay[e]) * ipy) * inv_n1;
        const double u = ua + du * (double)k[e];
        const double v = va + dv * (double)k[e];
        inside[e] = (u >= 0.0) & (u <= (double)(nx - 1)) & (v >= 0.0) & (v <= (double)(ny - 1));
        const double uc = inside[e] ? u : 0.0;   // in [0, nx - 1]: the conversion is defined
        const double vc = inside[e] ? v : 0.0;
        const int i = min((int)uc, nx - 2);      // uc >= 0: truncation is floor
        const int j = min((int)vc, ny - 2);
        fx[e] = uc - (double)i;
        fy[e] = vc - (double)j;
        const double *p = mu + (int64_t)j * nx + i;
        m00[e] = p[0];
        m01[e] = p[1];
        m10[e] = p[nx];
        m11[e] = p[nx + 1];
    }
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        const double r0v = m00[e] + fx[e] * (m01[e] - m00[e]);
        const double r1v = m10[e] + fx[e] * (m11[e] - m10[e]);
        const double val = r0v + fy[e] * (r1v - r0v);
        if (live[e]) __builtin_nontemporal_store(inside[e] ? val : __builtin_nan(""), out + t[e] * n_samples + k[e]);
    }
}

// Tracks of at least kWaveChunk / kSpt samples: each wave takes kWaveChunk
// consecutive samples of one track, so the track's end points are uniform
// (scalar loads) and its set-up in centre-index space is done once per
// wave; each lane then takes kSpt samples, 64 apart, and every store of the
// wave is 64 consecutive values.  The arithmetic of a sample is the same as
// light_curve_kernel's, operation for operation.
constexpr int kWaveChunk = 64 * kSpt;
typedef const __attribute__((address_space(4))) double ConstDouble;

// A value every lane of the wave holds alike, in scalar registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Eight waves per SIMD (at most 64 VGPRs): the gathers' latency is hidden
// by waves, not by work within one.
__global__ __launch_bounds__(kLcThreads, 8) void light_curve_track_kernel(
    const double *__restrict__ mu, int nx, int ny, double x0, double y0, double ipx, double ipy,
    const double *__restrict__ xa, const double *__restrict__ ya, const double *__restrict__ xb,
    const double *__restrict__ yb, const int32_t *__restrict__ order, const double *__restrict__ sorted,
    int64_t n_tracks, int64_t n_chunks, int chunks_per_track, int n_samples, double inv_n1,
    double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t chunk = wave_uniform((int64_t)blockIdx.x * (kLcThreads / 64) + threadIdx.x / 64);
    if (chunk >= n_chunks) return;   // uniform in the wave
    const int64_t tp = chunk / chunks_per_track;
    const int k0 = (int)(chunk - tp * chunks_per_track) * kWaveChunk;
    int64_t t = tp;
    double ax, ay, bx, by;
    if (order) {
        t = ((const __attribute__((address_space(4))) int32_t *)order)[tp];
        if (sorted) {   // end points in visiting order: read beside the order, not after it
            const ConstDouble *cs = (const ConstDouble *)sorted;
            ax = cs[tp];
            ay = cs[n_tracks + tp];
            bx = cs[2 * n_tracks + tp];
            by = cs[3 * n_tracks + tp];
        }
        if (t < 0 || t >= n_tracks) return;   // uniform: entries outside the tracks are skipped
    }
    if (!sorted) {
        const ConstDouble *cxa = (const ConstDouble *)xa, *cya = (const ConstDouble *)ya;
        const ConstDouble *cxb = (const ConstDouble *)xb, *cyb = (const ConstDouble *)yb;
        ax = cxa[t];
        ay = cya[t];
        bx = cxb[t];
        by = cyb[t];
    }
    const int lane = threadIdx.x % 64;
    const double ua = (ax - x0) * ipx - 0.5;
    const double va = (ay - y0) * ipy - 0.5;
    const double du = ((bx - ax) * ipx) * inv_n1;
    const double dv = ((by - ay) * ipy) * inv_n1;
    double fx[kSpt], fy[kSpt], m00[kSpt], m01[kSpt], m10[kSpt], m11[kSpt];
    bool inside[kSpt];
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        const int k = k0 + lane + 64 * e;
        const double u = ua + du * (double)k;
        const double v = va + dv * (double)k;
        inside[e] = (u >= 0.0) & (u <= (double)(nx - 1)) & (v >= 0.0) & (v <= (double)(ny - 1));
        const double uc = inside[e] ? u : 0.0;   // in [0, nx - 1]: the conversion is defined
        const double vc = inside[e] ? v : 0.0;
        const int i = min((int)uc, nx - 2);      // uc >= 0: truncation is floor
        const int j = min((int)vc, ny - 2);
        fx[e] = uc - (double)i;
        fy[e] = vc - (double)j;
        const double *p = mu + (int64_t)j * nx + i;
        m00[e] = p[0];
        m01[e] = p[1];
        m10[e] = p[nx];
        m11[e] = p[nx + 1];
    }
    double *row = out + t * n_samples;
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        const int k = k0 + lane + 64 * e;
        const double r0v = m00[e] + fx[e] * (m01[e] - m00[e]);
        const double r1v = m10[e] + fx[e] * (m11[e] - m10[e]);
        const double val = r0v + fy[e] * (r1v - r0v);
        if (k < n_samples) __builtin_nontemporal_store(inside[e] ? val : __builtin_nan(""), row + k);
    }
}

// --- track order: a counting sort of the tracks by the cell holding their
// midpoint, cells of kCellPx x kCellPx pixels (larger for maps of more than
// 2048 cells a side) numbered in Z (Morton) order, so that tracks that run
// together on the GPU read neighbouring parts of the map.
constexpr int kCellPx = 16;
constexpr int kMaxCellsPerSide = 2048;
constexpr int kScanThreads = 1024;

// Cell counters one 128-byte cache line apart while there are few cells:
// every track of a cell adds to its counter, and atomics on one line are
// served one after another (with 4096 cells, 32 counters a line took 256 x
// 32 atomics each).  Beyond 32768 cells the tracks spread over enough lines.
inline int counter_stride(int64_t n_keys) { return n_keys <= 32768 ? 32 : 1; }

struct CellGrid {
    double x0, y0, ipx, ipy;   // map origin and inverse pixel size
    int cell_px;               // pixels per cell side
    int cells_x, cells_y;
    int side;                  // power of two >= cells_x, cells_y
};

CellGrid cell_grid(const raysh_pixels *g) {
    CellGrid c{};
    c.x0 = g->x0;
    c.y0 = g->y0;
    c.ipx = 1.0 / g->px;
    c.ipy = 1.0 / g->py;
    c.cell_px = kCellPx;
    while ((std::max(g->nx, g->ny) + c.cell_px - 1) / c.cell_px > kMaxCellsPerSide) c.cell_px *= 2;
    c.cells_x = (g->nx + c.cell_px - 1) / c.cell_px;
    c.cells_y = (g->ny + c.cell_px - 1) / c.cell_px;
    c.side = 1;
    while (c.side < c.cells_x || c.side < c.cells_y) c.side *= 2;
    return c;
}

__device__ __forceinline__ int cell_of(double coord, int cells) {
    // coord in cells; NaN and values below 0 go to cell 0, values beyond the map to the last cell
    if (!(coord >= 0.0)) return 0;
    if (coord >= (double)cells) return cells - 1;
    return (int)coord;
}

__device__ __forceinline__ uint32_t morton(uint32_t x, uint32_t y) {
    uint32_t key = 0;
    for (int b = 0; b < 12; ++b) key |= ((x >> b) & 1u) << (2 * b) | ((y >> b) & 1u) << (2 * b + 1);
    return key;
}

// The counting and the scattering pass must agree on every key: the same
// operations, none contracted.
__device__ __forceinline__ uint32_t track_key(const CellGrid &c, double xa, double ya, double xb, double yb) {
#pragma clang fp contract(off)
    const double mx = 0.5 * (xa + xb), my = 0.5 * (ya + yb);
    const int cx = cell_of(((mx - c.x0) * c.ipx) / (double)c.cell_px, c.cells_x);
    const int cy = cell_of(((my - c.y0) * c.ipy) / (double)c.cell_px, c.cells_y);
    return morton((uint32_t)cx, (uint32_t)cy);
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(kLcThreads) void track_count_kernel(CellGrid c, const double *xa, const double *ya,
                                                                 const double *xb, const double *yb,
                                                                 int64_t n_tracks, int stride, uint32_t *counts) {
    const int64_t t = (int64_t)blockIdx.x * kLcThreads + threadIdx.x;
    if (t >= n_tracks) return;
    atomicAdd(&counts[(int64_t)track_key(c, xa[t], ya[t], xb[t], yb[t]) * stride], 1u);
}

// Exclusive prefix sum of counts[0], counts[stride], ... (n values) in place
// (one workgroup): each thread sums a contiguous run, the runs' sums are
// scanned (within each wave by shuffles, then the waves' totals in turn),
// then each thread rewrites its run.
__global__ __launch_bounds__(kScanThreads) void track_scan_kernel(uint32_t *counts, int64_t n, int stride) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = std::min<int64_t>((int64_t)threadIdx.x * per, n);
    const int64_t hi = std::min<int64_t>(lo + per, n);
    uint32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += counts[i * stride];
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t up = __shfl_up(incl, off, 64);
        if (lane >= off) incl += up;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += wave_tot[w];
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = counts[i * stride];
        counts[i * stride] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kLcThreads) void track_scatter_kernel(CellGrid c, const double *xa, const double *ya,
                                                                   const double *xb, const double *yb,
                                                                   int64_t n_tracks, int stride, uint32_t *offsets,
                                                                   int32_t *order, double *sorted) {
    const int64_t t = (int64_t)blockIdx.x * kLcThreads + threadIdx.x;
    if (t >= n_tracks) return;
    const double ax = xa[t], ay = ya[t], bx = xb[t], by = yb[t];
    const uint32_t pos = atomicAdd(&offsets[(int64_t)track_key(c, ax, ay, bx, by) * stride], 1u);
    order[pos] = (int32_t)t;   // pos < n_tracks: the offsets partition [0, n_tracks)
    if (sorted) {
        sorted[pos] = ax;
        sorted[n_tracks + pos] = ay;
        sorted[2 * n_tracks + pos] = bx;
        sorted[3 * n_tracks + pos] = by;
    }
}

int check_profile(int profile, double size, double px, double py, int32_t nx, int32_t ny) {
    if (profile != RAYSH_SOURCE_GAUSSIAN && profile != RAYSH_SOURCE_DISK)
        return set_error(RAYSH_EINVAL, "unknown source profile %d", profile);
    if (nx <= 0 || ny <= 0) return set_error(RAYSH_EINVAL, "map size must be > 0");
    if (!(std::isfinite(size) && size > 0)) return set_error(RAYSH_EINVAL, "source size must be finite and > 0");
    if (!(std::isfinite(px) && px > 0) || !(std::isfinite(py) && py > 0))
        return set_error(RAYSH_EINVAL, "pixel size must be finite and > 0");
    const double reach = profile == RAYSH_SOURCE_GAUSSIAN ? 3.0 * size : size;
    if (!(reach / px < (double)nx) || !(reach / py < (double)ny))
        return set_error(RAYSH_EINVAL, "source larger than the map");
    return RAYSH_OK;
}

void radii(int profile, double size, double px, double py, int *rx, int *ry) {
    if (profile == RAYSH_SOURCE_GAUSSIAN) {
        *rx = taps_radius(size, px);
        *ry = taps_radius(size, py);
    } else {
        disk_radii(size, px, py, rx, ry);
    }
}

}  // namespace

extern "C" int raysh_source_map_shape(int32_t nx, int32_t ny, int profile, double size, double px, double py,
                                      int32_t *rx, int32_t *ry) {
    if (int r = check_profile(profile, size, px, py, nx, ny)) return r;
    int a = 0, b = 0;
    radii(profile, size, px, py, &a, &b);
    if (nx - 2 * a < 2 || ny - 2 * b < 2)
        return set_error(RAYSH_EINVAL, "the source map would have fewer than 2 x 2 pixels");
    if (rx) *rx = a;
    if (ry) *ry = b;
    return set_ok();
}

extern "C" size_t raysh_source_map_workspace(int32_t nx, int32_t ny) {
    if (nx <= 0 || ny <= 0) return 0;
    return 8 * ((size_t)nx * (size_t)ny + (size_t)nx + (size_t)ny + 4);
}

extern "C" int raysh_source_map(const int32_t *counts, int32_t nx, int32_t ny, double norm, int profile,
                                double size, double px, double py, void *workspace, size_t workspace_bytes,
                                double *mu_s, void *hip_stream) {
    int rx = 0, ry = 0;
    if (int r = raysh_source_map_shape(nx, ny, profile, size, px, py, &rx, &ry)) return r;
    if ((int64_t)nx * ny > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 pixels");
    if (!(std::isfinite(norm) && norm > 0)) return set_error(RAYSH_EINVAL, "norm must be finite and > 0");
    if (!counts || !workspace || !mu_s) return set_error(RAYSH_EINVAL, "NULL buffer");
    const size_t need = raysh_source_map_workspace(nx, ny);
    if (workspace_bytes < need)
        return set_error(RAYSH_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
    const int wx = nx - 2 * rx, wy = ny - 2 * ry;

    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, counts) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "counts is not device memory");
    }
    const int device = attr.device;
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    if (int r = validate_device_ptr(counts, (size_t)nx * ny * 4, device, "counts")) return r;
    if (int r = validate_device_ptr(workspace, need, device, "workspace")) return r;
    if (int r = validate_device_ptr(mu_s, (size_t)wx * wy * 8, device, "mu_s")) return r;

    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n_out = (int64_t)wx * wy;
    const unsigned blocks_out = (unsigned)((n_out + kLcThreads - 1) / kLcThreads);
    if (profile == RAYSH_SOURCE_GAUSSIAN) {
        double *tmp = (double *)workspace;                  // ny * wx
        double *gxt = tmp + (size_t)ny * wx;                // 2 rx + 1
        double *gyt = gxt + (2 * rx + 1);                   // 2 ry + 1
        hipLaunchKernelGGL(taps_kernel, dim3(1), dim3(kSmoothThreads), 0, s, size, px, rx, gxt);
        hipLaunchKernelGGL(taps_kernel, dim3(1), dim3(kSmoothThreads), 0, s, size, py, ry, gyt);
        const int64_t n1 = (int64_t)wx * ny;
        hipLaunchKernelGGL(smooth_rows_kernel, dim3((unsigned)((n1 + kSmoothThreads - 1) / kSmoothThreads)),
                           dim3(kSmoothThreads), 0, s, counts, nx, ny, norm, gxt, rx, wx, tmp);
        hipLaunchKernelGGL(smooth_cols_kernel, dim3(blocks_out), dim3(kSmoothThreads), 0, s, tmp, wx, wy, gyt,
                           ry, mu_s);
    } else {
        long long *n_taps = (long long *)workspace;
        int *half = (int *)(n_taps + 1);                    // 2 ry + 1 <= ny
        hipLaunchKernelGGL(disk_rows_kernel, dim3(1), dim3(kLcThreads), 0, s, size, px, py, rx, ry, half,
                           n_taps);
        hipLaunchKernelGGL(disk_map_kernel, dim3(blocks_out), dim3(kLcThreads), 0, s, counts, nx, norm, rx, ry,
                           half, n_taps, wx, wy, mu_s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_source_map");
    return set_ok();
}

extern "C" size_t raysh_track_order_workspace(const raysh_pixels *grid) {
    if (!grid || validate_pixels(grid) != RAYSH_OK) return 0;
    const CellGrid c = cell_grid(grid);
    const int64_t n_keys = (int64_t)c.side * c.side;
    return 4 * ((size_t)n_keys * (size_t)counter_stride(n_keys) + 1);
}

extern "C" int raysh_track_order(const raysh_pixels *grid, int64_t n_tracks, const double *xa, const double *ya,
                                 const double *xb, const double *yb, void *workspace, size_t workspace_bytes,
                                 int32_t *order, double *sorted, void *hip_stream) {
    if (!grid) return set_error(RAYSH_EINVAL, "raysh_track_order: grid is NULL");
    if (int r = validate_pixels(grid)) return r;
    if (n_tracks < 0) return set_error(RAYSH_EINVAL, "n_tracks < 0");
    if (n_tracks > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 tracks");
    if (n_tracks == 0) return set_ok();
    if (!xa || !ya || !xb || !yb || !order || !workspace) return set_error(RAYSH_EINVAL, "NULL buffer");
    const size_t need = raysh_track_order_workspace(grid);
    if (workspace_bytes < need)
        return set_error(RAYSH_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, xa) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "xa is not device memory");
    }
    const int device = attr.device;
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    const size_t tb = (size_t)n_tracks * 8;
    if (int r = validate_device_ptr(xa, tb, device, "xa")) return r;
    if (int r = validate_device_ptr(ya, tb, device, "ya")) return r;
    if (int r = validate_device_ptr(xb, tb, device, "xb")) return r;
    if (int r = validate_device_ptr(yb, tb, device, "yb")) return r;
    if (int r = validate_device_ptr(order, (size_t)n_tracks * 4, device, "order")) return r;
    if (sorted)
        if (int r = validate_device_ptr(sorted, (size_t)n_tracks * 32, device, "sorted")) return r;
    if (int r = validate_device_ptr(workspace, need, device, "workspace")) return r;

    hipStream_t s = (hipStream_t)hip_stream;
    const CellGrid c = cell_grid(grid);
    const int64_t n_keys = (int64_t)c.side * c.side;
    const int stride = counter_stride(n_keys);
    const int64_t n_words = n_keys * stride;
    uint32_t *counts = (uint32_t *)workspace;
    const unsigned tb_blocks = (unsigned)((n_tracks + kLcThreads - 1) / kLcThreads);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, s, counts, n_words);
    hipLaunchKernelGGL(track_count_kernel, dim3(tb_blocks), dim3(kLcThreads), 0, s, c, xa, ya, xb, yb, n_tracks,
                       stride, counts);
    hipLaunchKernelGGL(track_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, counts, n_keys, stride);
    hipLaunchKernelGGL(track_scatter_kernel, dim3(tb_blocks), dim3(kLcThreads), 0, s, c, xa, ya, xb, yb, n_tracks,
                       stride, counts, order, sorted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_track_order");
    return set_ok();
}

extern "C" int raysh_light_curves(const double *mu_s, const raysh_pixels *grid, int64_t n_tracks,
                                  int32_t n_samples, const double *xa, const double *ya, const double *xb,
                                  const double *yb, const int32_t *order, const double *sorted, double *curves,
                                  void *hip_stream) {
    if (!grid) return set_error(RAYSH_EINVAL, "raysh_light_curves: grid is NULL");
    if (int r = validate_pixels(grid)) return r;
    if (grid->nx < 2 || grid->ny < 2) return set_error(RAYSH_EINVAL, "the source map needs at least 2 x 2 pixels");
    if ((int64_t)grid->nx * grid->ny > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 pixels");
    if (n_tracks < 0) return set_error(RAYSH_EINVAL, "n_tracks < 0");
    if (n_samples < 1 || n_samples > (1 << 24)) return set_error(RAYSH_EINVAL, "n_samples outside [1, 2^24]");
    const int64_t max_total = (int64_t)std::numeric_limits<int32_t>::max() * (kSpt * kLcThreads);
    if (n_tracks > max_total / n_samples)
        return set_error(RAYSH_EOVERFLOW, "more than %lld samples", (long long)max_total);
    if (n_tracks == 0) return set_ok();
    if (!mu_s || !xa || !ya || !xb || !yb || !curves) return set_error(RAYSH_EINVAL, "NULL buffer");

    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, mu_s) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "mu_s is not device memory");
    }
    const int device = attr.device;
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    const size_t tb = (size_t)n_tracks * 8;
    if (int r = validate_device_ptr(mu_s, (size_t)grid->nx * grid->ny * 8, device, "mu_s")) return r;
    if (int r = validate_device_ptr(xa, tb, device, "xa")) return r;
    if (int r = validate_device_ptr(ya, tb, device, "ya")) return r;
    if (int r = validate_device_ptr(xb, tb, device, "xb")) return r;
    if (int r = validate_device_ptr(yb, tb, device, "yb")) return r;
    const int64_t total = n_tracks * (int64_t)n_samples;
    if (int r = validate_device_ptr(curves, (size_t)total * 8, device, "curves")) return r;
    if (order)
        if (int r = validate_device_ptr(order, (size_t)n_tracks * 4, device, "order")) return r;
    if (sorted && !order) return set_error(RAYSH_EINVAL, "sorted end points need their order");
    if (sorted)
        if (int r = validate_device_ptr(sorted, (size_t)n_tracks * 32, device, "sorted")) return r;

    hipStream_t s = (hipStream_t)hip_stream;
    const double inv_n1 = n_samples > 1 ? 1.0 / (double)(n_samples - 1) : 0.0;
    if (n_samples >= kWaveChunk / kSpt) {
        // one wave per kWaveChunk samples of a track
        const int chunks_per_track = (n_samples + kWaveChunk - 1) / kWaveChunk;
        const int64_t n_chunks = n_tracks * chunks_per_track;
        const int64_t waves_per_block = kLcThreads / 64;
        if ((n_chunks + waves_per_block - 1) / waves_per_block > std::numeric_limits<int32_t>::max())
            return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 workgroups of tracks");
        hipLaunchKernelGGL(light_curve_track_kernel,
                           dim3((unsigned)((n_chunks + waves_per_block - 1) / waves_per_block)), dim3(kLcThreads), 0,
                           s, mu_s, grid->nx, grid->ny, grid->x0, grid->y0, 1.0 / grid->px, 1.0 / grid->py, xa, ya, xb,
                           yb, order, sorted, n_tracks, n_chunks, chunks_per_track, n_samples, inv_n1, curves);
    } else {
        const float inv_nf = 1.0f / (float)n_samples;                   // n_samples <= 2^24: exact in float
        hipLaunchKernelGGL(light_curve_kernel,
                           dim3((unsigned)((total + kSpt * kLcThreads - 1) / (kSpt * kLcThreads))), dim3(kLcThreads),
                           0, s, mu_s, grid->nx, grid->ny, grid->x0, grid->y0, 1.0 / grid->px, 1.0 / grid->py, xa, ya,
                           xb, yb, order, sorted, n_tracks, n_samples, inv_nf, inv_n1, curves);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_light_curves");
    return set_ok();
}
