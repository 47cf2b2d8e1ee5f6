// Per-ray steps shared by the FP64 and FP32-bulk shooting kernels:
// the image angle, the macro term, beta -> pixel, and the LDS-windowed
// count accumulation (arXiv:1703.09707, Sec. 2.2, Algorithm 1).
#pragma once

#include "raysh_internal.h"

namespace raysh {

constexpr int kThreads = 256;   // 4 waves of 64
constexpr int kLanesX = 16;     // lanes of a workgroup along x
constexpr int kLanesY = 16;     // lanes of a workgroup along y
constexpr int kWinX = 64;       // LDS count window, pixels
constexpr int kWinY = 64;

// Cell-centred image angle: ((double)idx + 0.5) * step + origin, each
// operation rounded on its own (no contraction), as in the library's
// documented convention.
__device__ __forceinline__ double image_angle(double origin, int64_t idx, double step) {
#pragma clang fp contract(off)
    double t = (double)idx + 0.5;
    t = t * step;
    return origin + t;
}

// First term of Eq. (3): alpha_0 = K theta, without contraction.
__device__ __forceinline__ void macro_term(const ShootParams &p, double tx, double ty,
                                           double &ax, double &ay) {
#pragma clang fp contract(off)
    ax = p.k11 * tx + p.k12 * ty;
    ay = p.k12 * tx + p.k22 * ty;
}

// Eq. (2) and the pixel step of Algorithm 1: beta = theta - alpha, then the
// pixel coordinate (beta - X0) / P with IEEE division, the half-open window
// test in FP64, and floor.  Returns the linear index or -1.
__device__ __forceinline__ int32_t source_pixel(const ShootParams &p, double tx, double ty,
                                                double ax, double ay, double &bx, double &by,
                                                int32_t &is, int32_t &js) {
#pragma clang fp contract(off)
    bx = tx - ax;
    by = ty - ay;
    is = -1;
    js = -1;
    if (!__builtin_isfinite(bx) || !__builtin_isfinite(by)) return -1;
    const double u = (bx - p.X0) / p.Px;
    const double v = (by - p.Y0) / p.Py;
    if (!(u >= 0.0 && u < (double)p.NX && v >= 0.0 && v < (double)p.NY)) return -1;
    is = (int32_t)__builtin_floor(u);
    js = (int32_t)__builtin_floor(v);
    return js * p.NX + is;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Shared memory of the binning epilogue.
struct BinShared {
    int win[kWinY * kWinX];
    unsigned long long red[3];   // sum of is, sum of js, rays binned
};

__device__ __forceinline__ void bin_shared_init(BinShared &sh) {
    if (threadIdx.x < 3) sh.red[threadIdx.x] = 0;
}

// Epilogue of a ray tile: per-ray outputs, then the counts.  Each lane holds
// CX x CY rays: column a at block index i = tile_i + lx + 16 a, row b at
// j = tile_j + ly + 16 b.  Counts go first into an LDS window of WX x WY
// pixels (at most kWinX x kWinY) placed around the tile's mean pixel, with a
// global atomic for rays outside it; the window is then merged into the map
// with one global atomic per non-empty pixel.  With KEEP_CLEAR the window
// must be zero on entry and is left zero (the merge clears what it reads),
// which saves a pass over it for a caller that bins many tiles.  Must be
// reached by every thread of the workgroup (it contains barriers).
template <int CX, int CY, int WX = kWinX, int WY = kWinY, bool KEEP_CLEAR = false>
__device__ __forceinline__ void finish_tile(const ShootParams &p, BinShared &sh,
                                            const double (&tx)[CX], const double (&ty)[CY],
                                            const double (&ax)[CY][CX], const double (&ay)[CY][CX],
                                            int64_t tile_i, int64_t tile_j, int lx, int ly) {
    static_assert(WX > 0 && WY > 0 && WX * WY <= kWinX * kWinY, "the window fits BinShared");
    int32_t pis[CY][CX], pjs[CY][CX], pidx[CY][CX];
    long long s_is = 0, s_js = 0, n_in = 0;
#pragma unroll
    for (int b = 0; b < CY; ++b) {
#pragma unroll
        for (int a = 0; a < CX; ++a) {
            const int64_t i = tile_i + lx + kLanesX * a;
            const int64_t j = tile_j + ly + kLanesY * b;
            double bx, by;
            int32_t is, js;
            int32_t q = source_pixel(p, tx[a], ty[b], ax[b][a], ay[b][a], bx, by, is, js);
            const bool in_block = (i < p.nx) && (j < p.ny);
            if (in_block) {
                const int64_t o = j * p.nx + i;
                if (p.beta_x) p.beta_x[o] = bx;
                if (p.beta_y) p.beta_y[o] = by;
                if (p.bin) p.bin[o] = q;
            } else {
                q = -1;
            }
            pidx[b][a] = q;
            pis[b][a] = is;
            pjs[b][a] = js;
            if (q >= 0) {
                s_is += is;
                s_js += js;
                n_in += 1;
            }
        }
    }
    if (!p.counts) return;   // uniform: no barrier is skipped by part of the group

    s_is = wave_sum(s_is);
    s_js = wave_sum(s_js);
    n_in = wave_sum(n_in);
    if (!KEEP_CLEAR)
        for (int t = threadIdx.x; t < WX * WY; t += kThreads) sh.win[t] = 0;
    __syncthreads();   // red[] initialised at kernel start; win[] cleared
    if ((threadIdx.x & 63) == 0 && n_in > 0) {
        atomicAdd(&sh.red[0], (unsigned long long)s_is);
        atomicAdd(&sh.red[1], (unsigned long long)s_js);
        atomicAdd(&sh.red[2], (unsigned long long)n_in);
    }
    __syncthreads();
    const long long total = (long long)sh.red[2];
    if (total == 0) return;   // uniform
    const int ox = (int)((long long)sh.red[0] / total) - WX / 2;
    const int oy = (int)((long long)sh.red[1] / total) - WY / 2;
#pragma unroll
    for (int b = 0; b < CY; ++b) {
#pragma unroll
        for (int a = 0; a < CX; ++a) {
            if (pidx[b][a] < 0) continue;
            const unsigned wx = (unsigned)(pis[b][a] - ox);
            const unsigned wy = (unsigned)(pjs[b][a] - oy);
            if (wx < (unsigned)WX && wy < (unsigned)WY)
                atomicAdd(&sh.win[wy * WX + wx], 1);
            else
                atomicAdd(&p.counts[pidx[b][a]], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < WX * WY; t += kThreads) {
        const int v = sh.win[t];
        if (KEEP_CLEAR && v) sh.win[t] = 0;
        if (v) {
            const int gx = ox + (t % WX);
            const int gy = oy + (t / WX);
            if (gx >= 0 && gx < p.NX && gy >= 0 && gy < p.NY)
                atomicAdd(&p.counts[gy * p.NX + gx], v);
        }
    }
    if (threadIdx.x == 0 && p.n_binned) atomicAdd(p.n_binned, (unsigned long long)total);
}

// Star records read through the constant address space: no kernel writes
// them, and uniform loads from it become scalar loads whatever the kernel
// stores elsewhere.
typedef const __attribute__((address_space(4))) Star ConstStar;

__device__ __forceinline__ const ConstStar *const_stars(const Star *p) {
    return (const ConstStar *)p;
}

// A value every lane holds alike, moved to a scalar register.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double uniform_f64(double v) {
    return __builtin_bit_cast(double, uniform64(__builtin_bit_cast(int64_t, v)));
}

__device__ __forceinline__ const Star *uniform_ptr(const Star *p) {
    return (const Star *)(uintptr_t)uniform64((int64_t)(uintptr_t)p);
}

// Set owning queue item `item` (binary search over first_item; uniform).
__device__ __forceinline__ int find_set(const BatchArgs &b, int item) {
    int lo = 0, hi = b.n_sets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (b.sets[mid].first_item <= item) lo = mid;
        else hi = mid - 1;
    }
    return uniform(lo);
}

// Copy a set's parameters to LDS, one word per thread (the caller then
// waits at a barrier).
__device__ __forceinline__ void copy_set_to_lds(const BatchSet *src, BatchSet *dst) {
    static_assert(sizeof(BatchSet) % 4 == 0 && sizeof(BatchSet) / 4 <= kThreads,
                  "one word of BatchSet per thread");
    if (threadIdx.x < sizeof(BatchSet) / 4) {
        int w;
        __builtin_memcpy(&w, reinterpret_cast<const char *>(src) + 4 * threadIdx.x, 4);
        __builtin_memcpy(reinterpret_cast<char *>(dst) + 4 * threadIdx.x, &w, 4);
    }
}

}  // namespace raysh
