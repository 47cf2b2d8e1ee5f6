// Magnification map -> histogram of log10(mu_sigma / mu_ref), the data the
// learned surrogate is trained on.
//
// The ray count of a pixel is proportional to the magnification of a source
// there (arXiv:1703.09707, Sec. 1): mu = counts * norm with
// norm = (dx*dy)/(Px*Py).  A finite source sees the map convolved with its
// profile (Sec. 1); here a circular Gaussian of width sigma, sampled at pixel
// offsets |k| <= r = ceil(3 sigma / P), normalised per axis and applied
// separably (rows, then columns), keeping only pixels at least r from every
// edge.  Each smoothed pixel goes to one of nbins uniform bins of
// log10(mu_sigma / mu_ref) on [lo, hi), clamped to the end bins.
// Everything is FP64, so the bin decision is taken in FP64.
#include <cmath>
#include <limits>

#include "raysh_ctx.h"
#include "smooth.h"

namespace {

constexpr int kMaxBins = 4096;

// Column pass for pixel (i, j) of the valid interior, then its bin, counted
// in an LDS histogram and added to the global bin counts.
__global__ __launch_bounds__(kSmoothThreads) void smooth_cols_hist_kernel(
    const double *__restrict__ tmp, int wx, int wy, const double *__restrict__ gy, int ry, double mu_ref,
    int nbins, double lo, double hi, unsigned *__restrict__ bins) {
#pragma clang fp contract(off)
    __shared__ unsigned h[kMaxBins];
    for (int b = threadIdx.x; b < nbins; b += kSmoothThreads) h[b] = 0;
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
    if (idx < (int64_t)wx * wy) {
        const int j = (int)(idx / wx), i = (int)(idx % wx);
        const double *col = tmp + (int64_t)j * wx + i;
        double acc = 0.0;
        for (int k = 0; k <= 2 * ry; ++k) acc = acc + gy[k] * col[(int64_t)k * wx];
        int b = 0;
        if (acc > 0.0) {
            const double v = log10(acc / mu_ref);
            const double u = ((v - lo) / (hi - lo)) * (double)nbins;
            if (u >= (double)nbins) b = nbins - 1;
            else if (u > 0.0) b = (int)floor(u);
        }
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kSmoothThreads)
        if (h[b]) atomicAdd(&bins[b], h[b]);
}

__global__ void zero_bins_kernel(unsigned *bins, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bins[i] = 0;
}

__global__ void normalise_kernel(const unsigned *bins, int n, float *hist) {
    __shared__ unsigned long long total;
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int b = 0; b < n; ++b) t += bins[b];
        total = t;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n; b += blockDim.x)
        hist[b] = total ? (float)((double)bins[b] / (double)total) : 0.0f;
}


}  // namespace

extern "C" size_t raysh_histogram_workspace(int32_t nx, int32_t ny) {
    if (nx <= 0 || ny <= 0) return 0;
    return 8 * ((size_t)nx * (size_t)ny + (size_t)nx + (size_t)ny + 4);
}

extern "C" int raysh_log_mag_histogram(const int32_t *counts, int32_t nx, int32_t ny, double norm,
                                       double sigma, double px, double py, double mu_ref, int32_t nbins,
                                       double lo, double hi, void *workspace, size_t workspace_bytes,
                                       uint32_t *bin_counts, float *hist, void *hip_stream) {
    if (nx <= 0 || ny <= 0) return set_error(RAYSH_EINVAL, "map size must be > 0");
    if ((int64_t)nx * ny > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "more than 2^31-1 pixels");
    if (!(std::isfinite(norm) && norm > 0)) return set_error(RAYSH_EINVAL, "norm must be finite and > 0");
    if (!(std::isfinite(sigma) && sigma > 0)) return set_error(RAYSH_EINVAL, "sigma must be finite and > 0");
    if (!(std::isfinite(px) && px > 0) || !(std::isfinite(py) && py > 0))
        return set_error(RAYSH_EINVAL, "pixel size must be finite and > 0");
    if (!(std::isfinite(mu_ref) && mu_ref > 0)) return set_error(RAYSH_EINVAL, "mu_ref must be finite and > 0");
    if (nbins < 1 || nbins > kMaxBins) return set_error(RAYSH_EINVAL, "nbins must be in [1, %d]", kMaxBins);
    if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi))
        return set_error(RAYSH_EINVAL, "histogram range must be finite with lo < hi");
    if (3.0 * sigma / px > nx || 3.0 * sigma / py > ny)
        return set_error(RAYSH_EINVAL, "source (3 sigma) larger than the map");
    const int rx = taps_radius(sigma, px), ry = taps_radius(sigma, py);
    const int wx = nx - 2 * rx, wy = ny - 2 * ry;
    if (wx <= 0 || wy <= 0) return set_error(RAYSH_EINVAL, "no pixel lies 3 sigma inside the map");
    if (!counts || !workspace || !bin_counts) return set_error(RAYSH_EINVAL, "NULL buffer");
    if (workspace_bytes < raysh_histogram_workspace(nx, ny))
        return set_error(RAYSH_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes,
                         raysh_histogram_workspace(nx, ny));

    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, counts) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "counts is not device memory");
    }
    const int device = attr.device;
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    if (int r = validate_device_ptr(counts, (size_t)nx * ny * 4, device, "counts")) return r;
    if (int r = validate_device_ptr(workspace, raysh_histogram_workspace(nx, ny), device, "workspace"))
        return r;
    if (int r = validate_device_ptr(bin_counts, (size_t)nbins * 4, device, "bin_counts")) return r;
    if (hist)
        if (int r = validate_device_ptr(hist, (size_t)nbins * 4, device, "hist")) return r;

    hipStream_t s = (hipStream_t)hip_stream;
    double *tmp = (double *)workspace;                      // ny * wx
    double *gxt = tmp + (size_t)ny * wx;                    // 2 rx + 1
    double *gyt = gxt + (2 * rx + 1);                       // 2 ry + 1
    hipLaunchKernelGGL(taps_kernel, dim3(1), dim3(kSmoothThreads), 0, s, sigma, px, rx, gxt);
    hipLaunchKernelGGL(taps_kernel, dim3(1), dim3(kSmoothThreads), 0, s, sigma, py, ry, gyt);
    hipLaunchKernelGGL(zero_bins_kernel, dim3((nbins + 255) / 256), dim3(256), 0, s, bin_counts, nbins);
    const int64_t n1 = (int64_t)wx * ny, n2 = (int64_t)wx * wy;
    hipLaunchKernelGGL(smooth_rows_kernel, dim3((unsigned)((n1 + kSmoothThreads - 1) / kSmoothThreads)),
                       dim3(kSmoothThreads), 0, s, counts, nx, ny, norm, gxt, rx, wx, tmp);
    hipLaunchKernelGGL(smooth_cols_hist_kernel, dim3((unsigned)((n2 + kSmoothThreads - 1) / kSmoothThreads)),
                       dim3(kSmoothThreads), 0, s, tmp, wx, wy, gyt, ry, mu_ref, nbins, lo, hi,
                       (unsigned *)bin_counts);
    if (hist) hipLaunchKernelGGL(normalise_kernel, dim3(1), dim3(256), 0, s, (const unsigned *)bin_counts, nbins, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_log_mag_histogram");
    return set_ok();
}
