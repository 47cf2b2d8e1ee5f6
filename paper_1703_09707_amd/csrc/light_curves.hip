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
// plus the map read once.
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
    const double *__restrict__ yb, int64_t n_tracks, int n_samples, float inv_nf, double inv_n1,
    double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t base = (int64_t)blockIdx.x * (kSpt * kLcThreads);
    const int64_t total = n_tracks * (int64_t)n_samples;
    const int64_t t0 = base / n_samples;
    const int r0 = (int)(base - t0 * n_samples) + (int)threadIdx.x;
    int64_t t[kSpt];
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
        t[e] = live[e] ? t0 + q : 0;   // a finished lane reads track 0 and stores nothing
        k[e] = kk;
    }
    double ax[kSpt], ay[kSpt], bx[kSpt], by[kSpt];
#pragma unroll
    for (int e = 0; e < kSpt; ++e) {
        ax[e] = xa[t[e]];
        ay[e] = ya[t[e]];
        bx[e] = xb[t[e]];
        by[e] = yb[t[e]];
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
        if (live[e]) out[base + threadIdx.x + e * kLcThreads] = inside[e] ? val : __builtin_nan("");
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

extern "C" int raysh_light_curves(const double *mu_s, const raysh_pixels *grid, int64_t n_tracks,
                                  int32_t n_samples, const double *xa, const double *ya, const double *xb,
                                  const double *yb, double *curves, void *hip_stream) {
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

    hipStream_t s = (hipStream_t)hip_stream;
    const float inv_nf = 1.0f / (float)n_samples;                       // n_samples <= 2^24: exact in float
    const double inv_n1 = n_samples > 1 ? 1.0 / (double)(n_samples - 1) : 0.0;
    hipLaunchKernelGGL(light_curve_kernel, dim3((unsigned)((total + kSpt * kLcThreads - 1) / (kSpt * kLcThreads))),
                       dim3(kLcThreads), 0, s, mu_s, grid->nx, grid->ny, grid->x0, grid->y0, 1.0 / grid->px,
                       1.0 / grid->py, xa, ya, xb, yb, n_tracks, n_samples, inv_nf, inv_n1, curves);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_light_curves");
    return set_ok();
}
