// FP64 backward ray shooting on gfx950 (arXiv:1703.09707, Eq. (1)-(3) and
// Algorithm 1).
//
// One workgroup of 256 lanes owns a tile of (16 CX) x (16 CY) rays; each lane
// owns CX columns and CY rows of it, so the x offset theta_x - x_k is shared
// by the lane's CY rays of a column, and the y offset and its square by the
// CX rays of a row.  r^2 = (theta_x - x_k)^2 + (theta_y - y_k)^2 is one FMA
// per ray on those shared values.
//
// Stars are read in index order with uniform loads (every lane reads the
// same record), which the compiler turns into scalar loads: star data sits
// in SGPRs and feeds the vector ALU as a scalar operand, so it costs no
// VGPRs and no LDS traffic.
//
// The division m_k / r_k^2 of Eq. (3) uses the hardware reciprocal, which
// is good to about 2^-24, refined by one Newton step.  SHARE stars share one
// reciprocal: for two stars, y = 1 / (r_a^2 r_b^2) refined once, then
// 1/r_a^2 = r_b^2 y and 1/r_b^2 = r_a^2 y; four stars do the same with a
// product of four.  The relative error of each 1/r^2 is a few units in the
// last place of FP64 (the refined reciprocal is good to about 2^-48).  A ray
// exactly on a star gets a zero product, an infinite or NaN weight and a
// non-finite beta, and is dropped, as the plain definition drops it.
// The mass multiplies either the per-column and per-row offsets (when a lane
// owns more rays than it has rows plus columns) or 1/r^2 of each ray; the
// accumulation alpha += (m/r^2)(theta - theta_k) is one FMA per component,
// stars in index order.
#include "ray_common.h"

namespace raysh {

namespace {

// 1 / r2[s] for SHARE stars from one hardware reciprocal (good to about
// 2^-24) of their product, refined by one Newton step (to about 2^-48), then
// multiplied back by the other factors.
template <int SHARE>
__device__ __forceinline__ void reciprocals(const double (&r2)[SHARE], double (&inv)[SHARE]) {
    if constexpr (SHARE == 1) {
        double y = __builtin_amdgcn_rcp(r2[0]);
        const double e = __builtin_fma(-r2[0], y, 1.0);
        inv[0] = __builtin_fma(y, e, y);
    } else if constexpr (SHARE == 2) {
        const double pr = r2[0] * r2[1];
        double y = __builtin_amdgcn_rcp(pr);
        const double e = __builtin_fma(-pr, y, 1.0);
        y = __builtin_fma(y, e, y);
        inv[0] = r2[1] * y;
        inv[1] = r2[0] * y;
    } else {
        static_assert(SHARE == 4, "SHARE is 1, 2 or 4");
        const double p01 = r2[0] * r2[1];
        const double p23 = r2[2] * r2[3];
        const double pr = p01 * p23;
        double y = __builtin_amdgcn_rcp(pr);
        const double e = __builtin_fma(-pr, y, 1.0);
        y = __builtin_fma(y, e, y);
        const double y01 = p23 * y;   // 1 / (r0^2 r1^2)
        const double y23 = p01 * y;   // 1 / (r2^2 r3^2)
        inv[0] = r2[1] * y01;
        inv[1] = r2[0] * y01;
        inv[2] = r2[3] * y23;
        inv[3] = r2[2] * y23;
    }
}

__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// One ray tile (all of Algorithm 1 for its rays).  sh.red must be zero on
// entry; every thread of the workgroup must call it.
template <int CX, int CY, int SHARE>
__device__ __forceinline__ void fp64_tile(const ShootParams &p, BinShared &sh, int64_t tile) {
    // Fold the mass into the per-column and per-row offsets when that takes
    // fewer multiplies (CX + CY per star) than weighting every ray (CX * CY).
    constexpr bool FOLD = CX * CY > CX + CY;
    const int lx = threadIdx.x % kLanesX;
    const int ly = threadIdx.x / kLanesX;
    const int64_t tile_i = (tile % p.tiles_x) * (kLanesX * CX);
    const int64_t tile_j = (tile / p.tiles_x) * (kLanesY * CY);

    double tx[CX], ty[CY];
#pragma unroll
    for (int a = 0; a < CX; ++a) tx[a] = image_angle(p.x0, p.i0 + tile_i + lx + kLanesX * a, p.dx);
#pragma unroll
    for (int b = 0; b < CY; ++b) ty[b] = image_angle(p.y0, p.j0 + tile_j + ly + kLanesY * b, p.dy);

    double ax[CY][CX], ay[CY][CX];
#pragma unroll
    for (int b = 0; b < CY; ++b)
#pragma unroll
        for (int a = 0; a < CX; ++a) macro_term(p, tx[a], ty[b], ax[b][a], ay[b][a]);

    const Star *__restrict__ st = p.stars;
    const int n = p.n_stars;
    int k = 0;
    // star groups are double-buffered: the next group's scalar loads are in
    // flight while the current group is computed (the index of the group
    // after the last stays on the last, so every load is in bounds)
    double sx[SHARE], sy[SHARE], sm[SHARE];
    if (n >= SHARE) {
#pragma unroll
        for (int s = 0; s < SHARE; ++s) {
            sx[s] = st[s].x;
            sy[s] = st[s].y;
            sm[s] = st[s].m;
        }
    }
    for (; k + SHARE <= n; k += SHARE) {
        const int kn = (k + 2 * SHARE <= n) ? k + SHARE : k;
        double nx[SHARE], ny[SHARE], nm[SHARE];
#pragma unroll
        for (int s = 0; s < SHARE; ++s) {
            nx[s] = st[kn + s].x;
            ny[s] = st[kn + s].y;
            nm[s] = st[kn + s].m;
        }
        // per column: the x offset and (FOLD) the offset times the mass;
        // per row: the square of the y offset and the y offset (times the mass)
        double ex[SHARE][CX], mex[SHARE][CX], ey2[SHARE][CY], mey[SHARE][CY];
#pragma unroll
        for (int s = 0; s < SHARE; ++s) {
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                ex[s][a] = tx[a] - sx[s];
                mex[s][a] = FOLD ? sm[s] * ex[s][a] : ex[s][a];
            }
#pragma unroll
            for (int b = 0; b < CY; ++b) {
                const double e = ty[b] - sy[s];
                ey2[s][b] = mul_rn(e, e);
                mey[s][b] = FOLD ? sm[s] * e : e;
            }
        }
#pragma unroll
        for (int b = 0; b < CY; ++b) {
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                double r2[SHARE], inv[SHARE];
#pragma unroll
                for (int s = 0; s < SHARE; ++s) r2[s] = __builtin_fma(ex[s][a], ex[s][a], ey2[s][b]);
                reciprocals<SHARE>(r2, inv);
#pragma unroll
                for (int s = 0; s < SHARE; ++s) {
                    const double w = FOLD ? inv[s] : sm[s] * inv[s];
                    ax[b][a] = __builtin_fma(w, mex[s][a], ax[b][a]);
                    ay[b][a] = __builtin_fma(w, mey[s][b], ay[b][a]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < SHARE; ++s) {
            sx[s] = nx[s];
            sy[s] = ny[s];
            sm[s] = nm[s];
        }
    }
    for (; k < n; ++k) {   // remaining stars, one at a time, still in index order
        const double sx = st[k].x, sy = st[k].y, sm = st[k].m;
#pragma unroll
        for (int b = 0; b < CY; ++b) {
            const double ey = ty[b] - sy;
            const double ey2 = mul_rn(ey, ey);
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                const double ex = tx[a] - sx;
                double r2[1] = {__builtin_fma(ex, ex, ey2)}, inv[1];
                reciprocals<1>(r2, inv);
                const double w = sm * inv[0];
                ax[b][a] = __builtin_fma(w, ex, ax[b][a]);
                ay[b][a] = __builtin_fma(w, ey, ay[b][a]);
            }
        }
    }

    finish_tile<CX, CY>(p, sh, tx, ty, ax, ay, tile_i, tile_j, lx, ly);
}

template <int CX, int CY, int SHARE>
__global__ __launch_bounds__(kThreads) void shoot_fp64_kernel(ShootParams p) {
    __shared__ BinShared sh;
    bin_shared_init(sh);
    fp64_tile<CX, CY, SHARE>(p, sh, blockIdx.x);
}

// Persistent form: workgroups take (set, tile) items from a device queue
// until it is empty.
template <int CX, int CY, int SHARE>
__global__ __launch_bounds__(kThreads) void batch_fp64_kernel(BatchArgs b) {
    __shared__ BinShared sh;
    __shared__ long long s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(b.queue, 1ull);
        bin_shared_init(sh);
        __syncthreads();
        const long long item = s_item;
        if (item >= b.total_items) break;   // uniform: every wave leaves
        const int set = find_set(b, item);
        const BatchSet &bs = b.sets[set];
        const int64_t t0 = (item - bs.first_item) * bs.tiles_per_item;
        const int64_t t1 = t0 + bs.tiles_per_item < bs.n_tiles ? t0 + bs.tiles_per_item : bs.n_tiles;
        for (int64_t t = t0; t < t1; ++t) {   // uniform trip count
            fp64_tile<CX, CY, SHARE>(bs.p, sh, t);
            __syncthreads();   // red and the window are reused
            bin_shared_init(sh);
        }
        __syncthreads();   // s_item is rewritten
    }
}

template <int CX, int CY, int SHARE>
hipError_t launch_batch(const BatchArgs &b, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((batch_fp64_kernel<CX, CY, SHARE>), dim3(blocks), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

template <int CX, int CY, int SHARE>
int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_fp64_kernel<CX, CY, SHARE>, kThreads, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int CX, int CY, int SHARE>
hipError_t launch(const ShootParams &p, hipStream_t s) {
    const int64_t tiles_y = (p.ny + kLanesY * CY - 1) / (kLanesY * CY);
    ShootParams q = p;
    q.tiles_x = (int32_t)((p.nx + kLanesX * CX - 1) / (kLanesX * CX));
    const int64_t blocks = (int64_t)q.tiles_x * tiles_y;
    hipLaunchKernelGGL((shoot_fp64_kernel<CX, CY, SHARE>), dim3((unsigned)blocks), dim3(kThreads),
                       0, s, q);
    return hipGetLastError();
}

}  // namespace

#define RAYSH_FP64_SHAPES(X) \
    X(1, 4, 2)               \
    X(2, 2, 2)               \
    X(2, 4, 1)               \
    X(2, 4, 2)               \
    X(2, 4, 4)               \
    X(4, 2, 4)               \
    X(4, 4, 2)               \
    X(4, 4, 4)               \
    X(2, 8, 2)               \
    X(2, 8, 4)

int fp64_shape_list(TileShape *out, int cap) {
    int n = 0;
#define RAYSH_CASE(CX, CY, S)                          \
    if (n < cap) out[n] = TileShape{CX, CY, S, 0}; \
    ++n;
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return n;
}

bool fp64_shape_supported(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.share == S) return true;
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return false;
}

hipError_t launch_shoot_fp64(const ShootParams &p, const TileShape &t, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.share == S) return launch<CX, CY, S>(p, s);
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch_fp64(const BatchArgs &b, const TileShape &t, int blocks, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.share == S) return launch_batch<CX, CY, S>(b, blocks, s);
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

int batch_fp64_blocks_per_cu(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.share == S) return batch_blocks_per_cu<CX, CY, S>();
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return 1;
}

int tile_width(const TileShape &t) { return kLanesX * t.cx; }
int tile_height(const TileShape &t) { return kLanesY * t.cy; }

namespace {
__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
}  // namespace

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace raysh
