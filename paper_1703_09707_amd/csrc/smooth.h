// Separable Gaussian smoothing of a count map, shared by the log-magnification
// histogram and the source maps of light curves.
//
// A source of finite size sees the magnification map convolved with its
// profile (arXiv:1703.09707, Sec. 1).  For a circular Gaussian of width sigma
// the profile is sampled at pixel offsets |k| <= r = ceil(3 sigma / P),
// normalised per axis, and applied rows first, then columns, in FP64 with
// every product and sum rounded on its own.  Only pixels at least r from
// every edge are kept.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

namespace {

constexpr int kSmoothThreads = 256;

// taps[0..2r] of one axis: exp(-0.5 ((k - r) P / sigma)^2), then divided by
// their sum (one workgroup).
__global__ __launch_bounds__(kSmoothThreads) void taps_kernel(double sigma, double pixel, int r,
                                                            double *taps) {
    __shared__ double part[kSmoothThreads];
    const int n = 2 * r + 1;
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += kSmoothThreads) {
        const double d = ((double)(k - r) * pixel) / sigma;
        const double g = exp(-0.5 * (d * d));
        taps[k] = g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {   // sum in index order, as a plain loop does
        for (int k = 0; k < n; ++k) s += taps[k];
        part[0] = s;
    }
    __syncthreads();
    const double total = part[0];
    for (int k = threadIdx.x; k < n; k += kSmoothThreads) taps[k] = taps[k] / total;
}

// tmp[j][i] = sum_k gx[k] * (counts[j][i + k] * norm), i < wx, taps in order.
__global__ __launch_bounds__(kSmoothThreads) void smooth_rows_kernel(const int32_t *__restrict__ counts,
                                                                   int nx, int ny, double norm,
                                                                   const double *__restrict__ gx,
                                                                   int rx, int wx, double *__restrict__ tmp) {
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
    if (idx >= (int64_t)wx * ny) return;
    const int j = (int)(idx / wx), i = (int)(idx % wx);
    const int32_t *row = counts + (int64_t)j * nx + i;
    double acc = 0.0;
    for (int k = 0; k <= 2 * rx; ++k) acc = acc + gx[k] * ((double)row[k] * norm);
    tmp[idx] = acc;
}

// out[j][i] = sum_l gy[l] * tmp[j + l][i] over the valid interior.
__global__ __launch_bounds__(kSmoothThreads) void smooth_cols_kernel(const double *__restrict__ tmp, int wx,
                                                                     int wy, const double *__restrict__ gy,
                                                                     int ry, double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
    if (idx >= (int64_t)wx * wy) return;
    const int j = (int)(idx / wx), i = (int)(idx % wx);
    const double *col = tmp + (int64_t)j * wx + i;
    double acc = 0.0;
    for (int k = 0; k <= 2 * ry; ++k) acc = acc + gy[k] * col[(int64_t)k * wx];
    out[idx] = acc;
}

inline int taps_radius(double sigma, double pixel) { return (int)std::ceil(3.0 * sigma / pixel); }

}  // namespace
