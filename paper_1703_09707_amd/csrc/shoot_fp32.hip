// FP32-bulk backward ray shooting on gfx950.
//
// Same rays, macro term and pixel step as the FP64 path (all FP64); only the
// star terms m_k (theta - theta_k) / |theta - theta_k|^2 of Eq. (3) are
// evaluated in FP32, on coordinates relative to the centre c of the
// workgroup's ray tile:
//   - each lane holds its ray offsets theta - c rounded to FP32;
//   - the workgroup stages S stars at a time in LDS as FP32 (x_k - c, y_k - c, m_k),
//     the differences taken in FP64 before rounding, so that stars near the
//     tile keep full FP32 relative accuracy;
//   - every lane reads each staged star as one LDS broadcast and forms the
//     term with FP32 FMAs and the hardware FP32 reciprocal (the mass
//     multiplies the per-column and per-row offsets when a lane owns more
//     rays than it has rows plus columns);
//   - the FP32 partial sums of one staged tile are added to FP64 sums before
//     the next tile, stars in index order throughout.
#include "ray_common.h"

namespace raysh {

namespace {

// One ray tile.  sh.red must be zero on entry; every thread of the
// workgroup must call it.
template <int CX, int CY, int S>
__device__ __forceinline__ void fp32_tile(const ShootParams &p, BinShared &sh, float4 *stage,
                                          int64_t tile) {
    static_assert(S <= kThreads, "one star per thread when staging");
    // mass folded into the per-column and per-row offsets when cheaper
    constexpr bool FOLD = CX * CY > CX + CY;
    const int lx = threadIdx.x % kLanesX;
    const int ly = threadIdx.x / kLanesX;
    const int64_t tile_i = (tile % p.tiles_x) * (kLanesX * CX);
    const int64_t tile_j = (tile / p.tiles_x) * (kLanesY * CY);

    // tile centre: the image angle of the tile's middle lattice point
    const double cx = image_angle(p.x0, p.i0 + tile_i + (kLanesX * CX) / 2, p.dx);
    const double cy = image_angle(p.y0, p.j0 + tile_j + (kLanesY * CY) / 2, p.dy);

    double tx[CX], ty[CY];
    float ox[CX], oy[CY];
#pragma unroll
    for (int a = 0; a < CX; ++a) {
        tx[a] = image_angle(p.x0, p.i0 + tile_i + lx + kLanesX * a, p.dx);
        ox[a] = (float)(tx[a] - cx);
    }
#pragma unroll
    for (int b = 0; b < CY; ++b) {
        ty[b] = image_angle(p.y0, p.j0 + tile_j + ly + kLanesY * b, p.dy);
        oy[b] = (float)(ty[b] - cy);
    }

    double ax[CY][CX], ay[CY][CX];
#pragma unroll
    for (int b = 0; b < CY; ++b)
#pragma unroll
        for (int a = 0; a < CX; ++a) macro_term(p, tx[a], ty[b], ax[b][a], ay[b][a]);

    const Star *__restrict__ st = uniform_ptr(p.stars);
    const int n = uniform(p.n_stars);
    for (int base = 0; base < n; base += S) {
        const int cnt = (n - base < S) ? (n - base) : S;
        if ((int)threadIdx.x < cnt) {
            const Star s = st[base + threadIdx.x];
            stage[threadIdx.x] = make_float4((float)(s.x - cx), (float)(s.y - cy), (float)s.m, 0.0f);
        }
        __syncthreads();
        float fx[CY][CX], fy[CY][CX];
#pragma unroll
        for (int b = 0; b < CY; ++b)
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                fx[b][a] = 0.0f;
                fy[b][a] = 0.0f;
            }
#pragma unroll 2
        for (int k = 0; k < cnt; ++k) {
            const float4 q = stage[k];
            float ex[CX], mex[CX], ey[CY], mey[CY], ey2[CY];
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                ex[a] = ox[a] - q.x;
                mex[a] = FOLD ? q.z * ex[a] : ex[a];
            }
#pragma unroll
            for (int b = 0; b < CY; ++b) {
                ey[b] = oy[b] - q.y;
                ey2[b] = ey[b] * ey[b];
                mey[b] = FOLD ? q.z * ey[b] : ey[b];
            }
#pragma unroll
            for (int b = 0; b < CY; ++b) {
#pragma unroll
                for (int a = 0; a < CX; ++a) {
                    const float r2 = __builtin_fmaf(ex[a], ex[a], ey2[b]);
                    const float inv = __builtin_amdgcn_rcpf(r2);
                    const float w = FOLD ? inv : q.z * inv;
                    fx[b][a] = __builtin_fmaf(w, mex[a], fx[b][a]);
                    fy[b][a] = __builtin_fmaf(w, mey[b], fy[b][a]);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < CY; ++b)
#pragma unroll
            for (int a = 0; a < CX; ++a) {
                ax[b][a] += (double)fx[b][a];
                ay[b][a] += (double)fy[b][a];
            }
        __syncthreads();   // the stage is rewritten next pass
    }

    finish_tile<CX, CY>(p, sh, tx, ty, ax, ay, tile_i, tile_j, lx, ly);
}

template <int CX, int CY, int S>
__global__ __launch_bounds__(kThreads) void shoot_fp32_kernel(ShootParams p) {
    __shared__ BinShared sh;
    __shared__ float4 stage[S];
    bin_shared_init(sh);
    fp32_tile<CX, CY, S>(p, sh, stage, blockIdx.x);
}

template <int CX, int CY, int S>
__global__ __launch_bounds__(kThreads) void batch_fp32_kernel(BatchArgs b) {
    __shared__ BinShared sh;
    __shared__ float4 stage[S];
    __shared__ BatchSet s_set;
    __shared__ long long s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(b.queue, 1ull);
        bin_shared_init(sh);
        __syncthreads();
        const long long item_all = s_item;
        if (item_all >= b.total_items) break;   // every wave reads the same value and leaves
        const int item = uniform((int)item_all);
        copy_set_to_lds(&b.sets[find_set(b, item)], &s_set);
        __syncthreads();
        const int64_t per = uniform(s_set.tiles_per_item);
        const int64_t t0 = (item - uniform64(s_set.first_item)) * per;
        const int64_t n_tiles = uniform64(s_set.n_tiles);
        const int64_t t1 = t0 + per < n_tiles ? t0 + per : n_tiles;
        for (int64_t t = t0; t < t1; ++t) {   // uniform trip count
            fp32_tile<CX, CY, S>(s_set.p, sh, stage, t);
            __syncthreads();   // red, the window and the stage are reused
            bin_shared_init(sh);
        }
        __syncthreads();   // s_item and s_set are rewritten
    }
}

template <int CX, int CY, int S>
hipError_t launch_batch(const BatchArgs &b, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((batch_fp32_kernel<CX, CY, S>), dim3(blocks), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

template <int CX, int CY, int S>
int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_fp32_kernel<CX, CY, S>, kThreads, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int CX, int CY, int S>
int shoot_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, shoot_fp32_kernel<CX, CY, S>, kThreads, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int CX, int CY, int S>
hipError_t launch(const ShootParams &p, hipStream_t s) {
    const int64_t tiles_y = (p.ny + kLanesY * CY - 1) / (kLanesY * CY);
    ShootParams q = p;
    q.tiles_x = (int32_t)((p.nx + kLanesX * CX - 1) / (kLanesX * CX));
    const int64_t blocks = (int64_t)q.tiles_x * tiles_y;
    hipLaunchKernelGGL((shoot_fp32_kernel<CX, CY, S>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       s, q);
    return hipGetLastError();
}

}  // namespace

#define RAYSH_FP32_SHAPES(X) \
    X(2, 2, 128)             \
    X(2, 4, 128)             \
    X(4, 4, 64)              \
    X(4, 4, 128)             \
    X(4, 4, 256)             \
    X(2, 8, 128)

int fp32_shape_list(TileShape *out, int cap) {
    int n = 0;
#define RAYSH_CASE(CX, CY, S)                          \
    if (n < cap) out[n] = TileShape{CX, CY, 0, S}; \
    ++n;
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return n;
}

bool fp32_shape_supported(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.star_tile == S) return true;
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return false;
}

hipError_t launch_shoot_fp32(const ShootParams &p, const TileShape &t, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.star_tile == S) return launch<CX, CY, S>(p, s);
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch_fp32(const BatchArgs &b, const TileShape &t, int blocks, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.star_tile == S) return launch_batch<CX, CY, S>(b, blocks, s);
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

int shoot_fp32_blocks_per_cu(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.star_tile == S) return shoot_blocks_per_cu<CX, CY, S>();
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return 1;
}

int batch_fp32_blocks_per_cu(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S) \
    if (t.cx == CX && t.cy == CY && t.star_tile == S) return batch_blocks_per_cu<CX, CY, S>();
    RAYSH_FP32_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return 1;
}

}  // namespace raysh
