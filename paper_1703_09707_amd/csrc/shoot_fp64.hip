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
// is good to about 2^-24 and issues at a quarter of the FMA rate, refined by
// one Newton step.  SHARE values of r^2 share one reciprocal: NS consecutive
// stars of one ray times GX x GY of the lane's rays (for instance one star
// and the eight rays of a lane row); 1/r^2 of each is recovered from the
// reciprocal of their product through a product tree (for two:
// y = 1/(r_a^2 r_b^2), 1/r_a^2 = r_b^2 y, 1/r_b^2 = r_a^2 y).  The relative
// error of each 1/r^2 is a few units in the last place of FP64 (the refined
// reciprocal is good to about 2^-48).  A ray exactly on a star makes the
// shared product zero and its partners' weights NaN, and separations far
// outside [1e-19, 1e19] take the product out of FP64 range; rays that end
// with a non-finite sum are therefore summed again one by one with a
// division per star, so that only a ray that sits on a star is dropped, as
// the plain definition drops it.
// The mass enters where it costs least: for groups of one star and several
// rays, at the root of the product tree (one multiply per group, and the
// leaves receive m/r^2); otherwise in the per-column and per-row offsets
// when a lane owns more rays than it has rows plus columns, else in 1/r^2
// of each ray.  The accumulation alpha += (m/r^2)(theta - theta_k) is one
// FMA per component, stars in index order.
#include "ray_common.h"

namespace raysh {

namespace {

// 1 / r[i] for N values from one hardware reciprocal (good to about 2^-24)
// of their product, refined by one Newton step (to about 2^-48).  The
// product is built as a balanced tree (N - 1 multiplies); walking the tree
// back down, each node's inverse times its sibling's product is the inverse
// of the node's other child (2 multiplies per node), so the leaves receive
// 1 / r[i].  Cost: 3 (N - 1) multiplies, one reciprocal, two FMAs.
template <int N>
__device__ __forceinline__ double tree_product(const double *r) {
    if constexpr (N == 1) return r[0];
    else return tree_product<N / 2>(r) * tree_product<N / 2>(r + N / 2);
}

template <int N>
__device__ __forceinline__ void tree_inverse(const double *r, double y, double *inv) {
    if constexpr (N == 1) {
        inv[0] = y;
    } else {
        const double lo = tree_product<N / 2>(r);       // common subexpressions of the up-sweep
        const double hi = tree_product<N / 2>(r + N / 2);
        tree_inverse<N / 2>(r, hi * y, inv);           // 1 / (product of the lower half)
        tree_inverse<N / 2>(r + N / 2, lo * y, inv + N / 2);
    }
}

template <int N>
__device__ __forceinline__ void reciprocals(const double *r, double *inv) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "N is a power of two");
    const double pr = tree_product<N>(r);
    double y = __builtin_amdgcn_rcp(pr);
    const double e = __builtin_fma(-pr, y, 1.0);
    y = __builtin_fma(y, e, y);
    tree_inverse<N>(r, y, inv);
}

// m / r[i] for N values that share the numerator m: the root's inverse is
// scaled by m inside its Newton step (t = m y, then t + t e with
// e = 1 - p y), so the leaves receive m / r[i] for one multiply per group.
template <int N>
__device__ __forceinline__ void scaled_reciprocals(const double *r, double m, double *inv) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "N is a power of two");
    const double pr = tree_product<N>(r);
    const double y = __builtin_amdgcn_rcp(pr);
    const double e = __builtin_fma(-pr, y, 1.0);
    const double t = m * y;
    tree_inverse<N>(r, __builtin_fma(t, e, t), inv);
}

__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// How the SHARE values of r^2 that share one reciprocal are chosen: NS
// consecutive stars, times GX columns of the lane's rays, times GY rows.
template <int CX, int CY, int SHARE, int NS>
struct Grouping {
    static constexpr int GX = (SHARE / NS) < CX ? (SHARE / NS) : CX;
    static constexpr int GY = SHARE / (NS * GX);
    static_assert(NS >= 1 && NS <= 4 && NS * GX * GY == SHARE && CX % GX == 0 && CY % GY == 0,
                  "SHARE = NS stars x GX columns x GY rows of the lane's rays");
};

// The second term of Eq. (3) for stars [k0, k1) of a lane's CX x CY rays,
// added to (ax, ay) in star index order.  Each reciprocal is shared by NS
// consecutive stars times GX x GY of the lane's rays.
template <int CX, int CY, int NS, int GX, int GY>
__device__ __forceinline__ void star_sum(const ConstStar *st, int k0, int k1, const double (&tx)[CX],
                                         const double (&ty)[CY], double (&ax)[CY][CX],
                                         double (&ay)[CY][CX]) {
    // Where the mass enters.  One star per group (NS = 1): the whole group
    // shares it, so it scales the group's root inverse (one multiply per
    // group).  Otherwise it is folded into the per-column and per-row
    // offsets when that takes fewer multiplies (CX + CY per star) than
    // weighting every ray (CX * CY).
    constexpr bool ROOT = NS == 1 && GX * GY > 1;
    constexpr bool FOLD = !ROOT && CX * CY > CX + CY;
    constexpr int G = NS * GX * GY;
    int k = k0;
    // star groups are double-buffered: the next group's scalar loads are in
    // flight while the current group is computed (the index of the group
    // after the last stays on the last, so every load is in bounds)
    double sx[NS], sy[NS], sm[NS];
    if (k + NS <= k1) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            asm volatile("" : "=s"(sx[s]) : "0"(st[k + s].x));
            asm volatile("" : "=s"(sy[s]) : "0"(st[k + s].y));
            asm volatile("" : "=s"(sm[s]) : "0"(st[k + s].m));
        }
    }
    for (; k + NS <= k1; k += NS) {
        const int kn = (k + 2 * NS <= k1) ? k + NS : k;
        double nx[NS], ny[NS], nm[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            nx[s] = st[kn + s].x;
            ny[s] = st[kn + s].y;
            nm[s] = st[kn + s].m;
        }
        __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the body
        // per column: the x offset and (FOLD) the offset times the mass;
        // per row: the square of the y offset and the y offset (times the mass)
        double ex[NS][CX], mex[NS][CX], ey2[NS][CY], mey[NS][CY];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
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
        for (int b0 = 0; b0 < CY; b0 += GY) {
#pragma unroll
            for (int a0 = 0; a0 < CX; a0 += GX) {
                // GX x GY rays of the lane and NS stars share one reciprocal
                double r2[G], inv[G];
#pragma unroll
                for (int gy = 0; gy < GY; ++gy)
#pragma unroll
                    for (int gx = 0; gx < GX; ++gx)
#pragma unroll
                        for (int s = 0; s < NS; ++s)
                            r2[(gy * GX + gx) * NS + s] =
                                __builtin_fma(ex[s][a0 + gx], ex[s][a0 + gx], ey2[s][b0 + gy]);
                if constexpr (ROOT) scaled_reciprocals<G>(r2, sm[0], inv);
                else reciprocals<G>(r2, inv);
#pragma unroll
                for (int gy = 0; gy < GY; ++gy) {
#pragma unroll
                    for (int gx = 0; gx < GX; ++gx) {
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            const int a = a0 + gx, b = b0 + gy;
                            const double inv1 = inv[(gy * GX + gx) * NS + s];
                            const double w = (FOLD || ROOT) ? inv1 : sm[s] * inv1;
                            ax[b][a] = __builtin_fma(w, mex[s][a], ax[b][a]);
                            ay[b][a] = __builtin_fma(w, mey[s][b], ay[b][a]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // an opaque hand-over: the prefetched records must be in their
            // scalar registers here, at the end of the body, and cannot be
            // reloaded next to their first use
            asm volatile("" : "=s"(sx[s]) : "0"(nx[s]));
            asm volatile("" : "=s"(sy[s]) : "0"(ny[s]));
            asm volatile("" : "=s"(sm[s]) : "0"(nm[s]));
        }
    }
    if constexpr (NS > 1) {
        for (; k < k1; ++k) {   // remaining stars, one at a time, still in index order
            const double sx1 = st[k].x, sy1 = st[k].y, sm1 = st[k].m;
#pragma unroll
            for (int b = 0; b < CY; ++b) {
                const double ey = ty[b] - sy1;
                const double ey2 = mul_rn(ey, ey);
#pragma unroll
                for (int a = 0; a < CX; ++a) {
                    const double ex = tx[a] - sx1;
                    double r2[1] = {__builtin_fma(ex, ex, ey2)}, inv[1];
                    reciprocals<1>(r2, inv);
                    const double w = sm1 * inv[0];
                    ax[b][a] = __builtin_fma(w, ex, ax[b][a]);
                    ay[b][a] = __builtin_fma(w, ey, ay[b][a]);
                }
            }
        }
    }
}

// True in every lane of the wave when any lane holds a non-finite sum.
template <int CX, int CY>
__device__ __forceinline__ bool wave_any_nonfinite(const double (&ax)[CY][CX], const double (&ay)[CY][CX]) {
    bool bad = false;
#pragma unroll
    for (int b = 0; b < CY; ++b)
#pragma unroll
        for (int a = 0; a < CX; ++a) bad |= !__builtin_isfinite(ax[b][a]) || !__builtin_isfinite(ay[b][a]);
    return __builtin_amdgcn_ballot_w64(bad) != 0;
}

// Stars [k0, k1) of one ray, added to (ax, ay) in index order with an IEEE
// division per star (the cold path below).
__device__ __forceinline__ void direct_star_sum(const ConstStar *st, int k0, int k1, double tx, double ty,
                                                double &ax, double &ay) {
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        const double ex = tx - st[k].x, ey = ty - st[k].y;
        const double w = st[k].m / __builtin_fma(ex, ex, mul_rn(ey, ey));
        ax = __builtin_fma(w, ex, ax);
        ay = __builtin_fma(w, ey, ay);
    }
}

// Stars [k0, k1) of the lane's rays, added to (ax, ay), which hold the macro
// term K theta (MACRO: one pass) or zero (a part of a split sum).  When
// several rays share a reciprocal, a ray exactly on a star (r^2 = 0) turns
// the shared product into zero and the weights of its partners into NaN, and
// separations beyond the product's FP64 range do the same.  So every ray that
// ends with a non-finite sum is summed again on its own, with a division per
// star: then only a ray that sits on a star stays non-finite (and is dropped,
// as in the definition).  That cold path goes through a private array indexed
// at run time, so that it claims no registers of the main loop.
template <int CX, int CY, int SHARE, int NS, bool MACRO>
__device__ __forceinline__ void lane_star_sums(const ShootParams &p, const ConstStar *st, int k0, int k1,
                                               const double (&tx)[CX], const double (&ty)[CY],
                                               double (&ax)[CY][CX], double (&ay)[CY][CX]) {
    using Gr = Grouping<CX, CY, SHARE, NS>;
    star_sum<CX, CY, NS, Gr::GX, Gr::GY>(st, k0, k1, tx, ty, ax, ay);
    if constexpr (SHARE > 1) {
        if (wave_any_nonfinite<CX, CY>(ax, ay)) {   // uniform across the wave
            double sum[2][CY * CX], ptx[CX], pty[CY];
#pragma unroll
            for (int a = 0; a < CX; ++a) ptx[a] = tx[a];
#pragma unroll
            for (int b = 0; b < CY; ++b) pty[b] = ty[b];
#pragma unroll
            for (int b = 0; b < CY; ++b)
#pragma unroll
                for (int a = 0; a < CX; ++a) {
                    sum[0][b * CX + a] = ax[b][a];
                    sum[1][b * CX + a] = ay[b][a];
                }
#pragma unroll 1
            for (int r = 0; r < CX * CY; ++r) {
                if (!__builtin_isfinite(sum[0][r]) || !__builtin_isfinite(sum[1][r])) {
                    const double rx = ptx[r % CX], ry = pty[r / CX];
                    double x = 0.0, y = 0.0;
                    if constexpr (MACRO) macro_term(p, rx, ry, x, y);
                    direct_star_sum(st, k0, k1, rx, ry, x, y);
                    sum[0][r] = x;
                    sum[1][r] = y;
                }
            }
#pragma unroll
            for (int b = 0; b < CY; ++b)
#pragma unroll
                for (int a = 0; a < CX; ++a) {
                    ax[b][a] = sum[0][b * CX + a];
                    ay[b][a] = sum[1][b * CX + a];
                }
        }
    }
}

// Image angles of a lane's CX columns and CY rows in ray tile `tile`.
template <int CX, int CY>
__device__ __forceinline__ void tile_rays(const ShootParams &p, int64_t tile, double (&tx)[CX],
                                          double (&ty)[CY], int64_t &tile_i, int64_t &tile_j, int &lx,
                                          int &ly) {
    lx = threadIdx.x % kLanesX;
    ly = threadIdx.x / kLanesX;
    const int64_t tiles_x = uniform(p.tiles_x);
    tile_i = (tile % tiles_x) * (kLanesX * CX);
    tile_j = (tile / tiles_x) * (kLanesY * CY);
#pragma unroll
    for (int a = 0; a < CX; ++a) tx[a] = image_angle(p.x0, p.i0 + tile_i + lx + kLanesX * a, p.dx);
#pragma unroll
    for (int b = 0; b < CY; ++b) ty[b] = image_angle(p.y0, p.j0 + tile_j + ly + kLanesY * b, p.dy);
}

// One ray tile (all of Algorithm 1 for its rays).  sh.red must be zero on
// entry; every thread of the workgroup must call it.
template <int CX, int CY, int SHARE, int NS>
__device__ __forceinline__ void fp64_tile(const ShootParams &p, BinShared &sh, int64_t tile) {
    double tx[CX], ty[CY];
    int64_t tile_i, tile_j;
    int lx, ly;
    tile_rays<CX, CY>(p, tile, tx, ty, tile_i, tile_j, lx, ly);
    double ax[CY][CX], ay[CY][CX];
#pragma unroll
    for (int b = 0; b < CY; ++b)
#pragma unroll
        for (int a = 0; a < CX; ++a) macro_term(p, tx[a], ty[b], ax[b][a], ay[b][a]);
    lane_star_sums<CX, CY, SHARE, NS, true>(p, const_stars(uniform_ptr(p.stars)), 0, uniform(p.n_stars), tx, ty,
                                            ax, ay);
    finish_tile<CX, CY>(p, sh, tx, ty, ax, ay, tile_i, tile_j, lx, ly);
}

template <int CX, int CY, int SHARE, int NS>
__global__ __launch_bounds__(kThreads, 2) void shoot_fp64_kernel(ShootParams p) {
    __shared__ BinShared sh;
    bin_shared_init(sh);
    fp64_tile<CX, CY, SHARE, NS>(p, sh, blockIdx.x);
}

// Persistent form: workgroups take items (runs of ray tiles of one set)
// from a device queue until it is empty.  The item's set is staged in LDS;
// the values the star loop needs are moved to scalar registers.  At least
// two waves per SIMD are requested: the queue loop keeps a few more values
// live than one tile does, and the compiler would otherwise give up the
// second wave for them.
template <int CX, int CY, int SHARE, int NS>
__global__ __launch_bounds__(kThreads, 2) void batch_fp64_kernel(BatchArgs b) {
    __shared__ BinShared sh;
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
            fp64_tile<CX, CY, SHARE, NS>(s_set.p, sh, t);
            __syncthreads();   // red and the window are reused
            bin_shared_init(sh);
        }
        __syncthreads();   // s_item and s_set are rewritten
    }
}

// Split-K form for many stars and few rays (the star sum of one ray split
// across workgroups): block (part, tile) adds stars [part*chunk, ...) for
// the tile's rays into partial[part][ray] (FP64 pairs, ray = j*nx + i of
// the block).  Blocks are numbered part-major, so blocks running together
// share their stars in the caches.
template <int CX, int CY, int SHARE, int NS>
__global__ __launch_bounds__(kThreads, 2) void partial_fp64_kernel(ShootParams p, int64_t n_tiles, int chunk,
                                                                double2 *__restrict__ partial) {
    const int part = (int)(blockIdx.x / n_tiles);
    const int64_t tile = blockIdx.x % n_tiles;
    double tx[CX], ty[CY];
    int64_t tile_i, tile_j;
    int lx, ly;
    tile_rays<CX, CY>(p, tile, tx, ty, tile_i, tile_j, lx, ly);
    double ax[CY][CX], ay[CY][CX];
#pragma unroll
    for (int b = 0; b < CY; ++b)
#pragma unroll
        for (int a = 0; a < CX; ++a) ax[b][a] = ay[b][a] = 0.0;
    const int64_t n = uniform(p.n_stars);
    const int64_t first = (int64_t)part * chunk;
    const int k0 = (int)(first < n ? first : n);
    const int k1 = (int)(k0 + (int64_t)chunk < n ? k0 + (int64_t)chunk : n);
    lane_star_sums<CX, CY, SHARE, NS, false>(p, const_stars(uniform_ptr(p.stars)), k0, k1, tx, ty, ax, ay);
    const int64_t n_rays = p.nx * p.ny;
#pragma unroll
    for (int b = 0; b < CY; ++b) {
#pragma unroll
        for (int a = 0; a < CX; ++a) {
            const int64_t i = tile_i + lx + kLanesX * a;
            const int64_t j = tile_j + ly + kLanesY * b;
            if (i < p.nx && j < p.ny) partial[part * n_rays + j * p.nx + i] = make_double2(ax[b][a], ay[b][a]);
        }
    }
}

// Split-K, second step: for every ray, alpha = K theta, then the parts'
// partial sums added in part order; the total overwrites part 0's slot.
// One thread per ray, so that every compute unit takes part (a lattice of
// few rays is few tiles), with the loads of kSumAhead parts issued before
// their additions.
constexpr int kSumAhead = 8;

__global__ __launch_bounds__(kThreads) void sum_parts_kernel(ShootParams p, int parts,
                                                             double2 *__restrict__ partial) {
    const int64_t n_rays = p.nx * p.ny;
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n_rays) return;
    const int64_t j = r / p.nx, i = r - j * p.nx;
    double ax, ay;
    macro_term(p, image_angle(p.x0, p.i0 + i, p.dx), image_angle(p.y0, p.j0 + j, p.dy), ax, ay);
    int q = 0;
    for (; q + kSumAhead <= parts; q += kSumAhead) {
        double2 v[kSumAhead];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) v[u] = partial[(int64_t)(q + u) * n_rays + r];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            ax += v[u].x;
            ay += v[u].y;
        }
    }
    for (; q < parts; ++q) {
        const double2 v = partial[(int64_t)q * n_rays + r];
        ax += v.x;
        ay += v.y;
    }
    partial[r] = make_double2(ax, ay);
}

// Split-K, last step: each ray's alpha from sum_parts_kernel, then beta,
// pixel and counts as in one pass.
template <int CX, int CY>
__global__ __launch_bounds__(kThreads) void finish_fp64_kernel(ShootParams p, const double2 *__restrict__ alpha) {
    __shared__ BinShared sh;
    bin_shared_init(sh);
    double tx[CX], ty[CY];
    int64_t tile_i, tile_j;
    int lx, ly;
    tile_rays<CX, CY>(p, blockIdx.x, tx, ty, tile_i, tile_j, lx, ly);
    double ax[CY][CX], ay[CY][CX];
#pragma unroll
    for (int b = 0; b < CY; ++b) {
#pragma unroll
        for (int a = 0; a < CX; ++a) {
            const int64_t i = tile_i + lx + kLanesX * a;
            const int64_t j = tile_j + ly + kLanesY * b;
            if (i < p.nx && j < p.ny) {
                const double2 v = alpha[j * p.nx + i];
                ax[b][a] = v.x;
                ay[b][a] = v.y;
            } else {
                macro_term(p, tx[a], ty[b], ax[b][a], ay[b][a]);
            }
        }
    }
    finish_tile<CX, CY>(p, sh, tx, ty, ax, ay, tile_i, tile_j, lx, ly);
}

template <int CX, int CY, int SHARE, int NS>
hipError_t launch_batch(const BatchArgs &b, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((batch_fp64_kernel<CX, CY, SHARE, NS>), dim3(blocks), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

template <int CX, int CY, int SHARE, int NS>
int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_fp64_kernel<CX, CY, SHARE, NS>, kThreads, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int CX, int CY, int SHARE, int NS>
int shoot_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, shoot_fp64_kernel<CX, CY, SHARE, NS>, kThreads, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int CX, int CY, int SHARE, int NS>
hipError_t launch(const ShootParams &p, hipStream_t s) {
    const int64_t tiles_y = (p.ny + kLanesY * CY - 1) / (kLanesY * CY);
    ShootParams q = p;
    q.tiles_x = (int32_t)((p.nx + kLanesX * CX - 1) / (kLanesX * CX));
    const int64_t blocks = (int64_t)q.tiles_x * tiles_y;
    hipLaunchKernelGGL((shoot_fp64_kernel<CX, CY, SHARE, NS>), dim3((unsigned)blocks), dim3(kThreads),
                       0, s, q);
    return hipGetLastError();
}

template <int CX, int CY, int SHARE, int NS>
hipError_t launch_split(const ShootParams &p, int parts, double2 *partial, hipStream_t s) {
    ShootParams q = p;
    q.tiles_x = (int32_t)((p.nx + kLanesX * CX - 1) / (kLanesX * CX));
    const int64_t tiles_y = (p.ny + kLanesY * CY - 1) / (kLanesY * CY);
    const int64_t n_tiles = (int64_t)q.tiles_x * tiles_y;
    int chunk = (int)((p.n_stars + parts - 1) / parts);
    chunk = (chunk + NS - 1) / NS * NS;
    hipLaunchKernelGGL((partial_fp64_kernel<CX, CY, SHARE, NS>), dim3((unsigned)(n_tiles * parts)), dim3(kThreads),
                       0, s, q, n_tiles, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_rays = q.nx * q.ny;
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((n_rays + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       q, parts, (double2 *)partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((finish_fp64_kernel<CX, CY>), dim3((unsigned)n_tiles), dim3(kThreads), 0, s, q,
                       (const double2 *)partial);
    return hipGetLastError();
}

}  // namespace

// Compiled launch shapes (CX, CY, SHARE, NS): rays per lane along x and y,
// r^2 values per reciprocal, consecutive stars among them.
#define RAYSH_FP64_SHAPES(X) \
    X(1, 4, 2, 2)            \
    X(2, 2, 2, 2)            \
    X(2, 4, 4, 4)            \
    X(2, 4, 8, 4)            \
    X(4, 2, 4, 4)            \
    X(4, 2, 8, 4)            \
    X(4, 4, 2, 2)            \
    X(4, 4, 4, 4)            \
    X(4, 4, 8, 4)            \
    X(2, 8, 2, 2)            \
    X(4, 4, 8, 1)            \
    X(4, 4, 16, 1)           \
    X(8, 2, 8, 1)            \
    X(8, 4, 8, 1)            \
    X(4, 8, 8, 1)            \
    X(8, 4, 16, 1)           \
    X(8, 5, 8, 1)

int fp64_shape_list(TileShape *out, int cap) {
    int n = 0;
#define RAYSH_CASE(CX, CY, S, NS)                       \
    if (n < cap) out[n] = TileShape{CX, CY, S, NS}; \
    ++n;
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return n;
}

bool fp64_shape_supported(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S, NS) \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) return true;
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return false;
}

hipError_t launch_shoot_fp64(const ShootParams &p, const TileShape &t, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S, NS) \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) return launch<CX, CY, S, NS>(p, s);
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_split_fp64(const ShootParams &p, const TileShape &t, int parts, double2 *partial,
                             hipStream_t s) {
#define RAYSH_CASE(CX, CY, S, NS)                                          \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) \
        return launch_split<CX, CY, S, NS>(p, parts, partial, s);
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch_fp64(const BatchArgs &b, const TileShape &t, int blocks, hipStream_t s) {
#define RAYSH_CASE(CX, CY, S, NS)                                          \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) \
        return launch_batch<CX, CY, S, NS>(b, blocks, s);
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return hipErrorInvalidValue;
}

int shoot_fp64_blocks_per_cu(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S, NS)                                          \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) \
        return shoot_blocks_per_cu<CX, CY, S, NS>();
    RAYSH_FP64_SHAPES(RAYSH_CASE)
#undef RAYSH_CASE
    return 1;
}

int batch_fp64_blocks_per_cu(const TileShape &t) {
#define RAYSH_CASE(CX, CY, S, NS)                                          \
    if (t.cx == CX && t.cy == CY && t.share == S && t.star_tile == NS) \
        return batch_blocks_per_cu<CX, CY, S, NS>();
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
