// FP64 ray shooting with the far field of the star sum as local (Taylor)
// expansions; a faster route to the sum of Eq. (3) for many stars.
//
// In complex notation (z = theta_x + i theta_y) the star term of Eq. (3) is
// alpha_x - i alpha_y = f(z) = sum_k m_k / (z - z_k).  Around a centre c,
// for a star with |c - z_k| > |z - c|,
//   m_k / (z - z_k) = sum_{q>=0} m_k u_k (-u_k rho)^q s^q,  u_k = 1/(c - z_k),
// with s = (z - c) / rho, so the far stars of a region add up to one
// polynomial F(s) = sum_q B_q s^q (the scaling by the region's radius rho
// keeps every |B_q| below sum m_k |u_k| theta_open^q, whatever the lattice
// spacing).  A star is far when |c - z_k| > rho / theta_open, with rho the
// region's radius (centre to corner ray): then every ray of the region has
// |(z - c) / (c - z_k)| <= theta_open and truncating after kOrder terms
// leaves an error below theta_open^(kOrder+1) (1 + theta_open) /
// (1 - theta_open) times m_k / |z - z_k| per star (1.5e-15 for
// theta_open = 0.25).  Near stars are summed directly, in index order.  The
// paper cites hierarchical tree codes as the way to avoid the brute-force
// sum (Sec. 1); this is a two-level form of that idea, on the ray side,
// whose truncation error stays at the level of FP64 rounding.
//
// Two levels.  The lattice is cut into blocks of L x L ray tiles (a tile is
// 64 x 64 rays, 4 x 4 per lane as in the one-pass kernel).  One workgroup
// per block expands the stars far from the whole block once (every star is
// visited once per block, not once per tile), keeping the block's near
// stars in lists.  Then one workgroup per row of the block's tiles
// re-centres the block's polynomial on each of its tiles (the shift of a
// polynomial is exact algebra: no new truncation), and for each tile
//   * re-tests only the block's near stars: those far from the tile join
//     its polynomial, the rest are summed directly,
//   * evaluates the polynomial for its rays (Horner), adds the near stars
//     and bins the rays.
// With L = 1 the block is the tile and the second test is skipped.  If a
// block has more near stars than its lists hold, its tiles sum every star
// directly.
//
// The block pass is a kernel of its own (expansion_block_kernel), which
// leaves each block's polynomial and near lists in a workspace for the
// tile kernel (expansion_fp64_kernel); each runs at the occupancy its own
// registers allow.
//
// Star cells.  Optionally the stars are sorted once by the cell of a
// regular grid, and each cell gets a multipole expansion of its stars
// (M_j = sum_k m_k ((z_k - z_c) / r_c)^j).  The block pass then takes every
// cell far enough from the block, (r_c + rho) / theta_open or more between
// centres, through one multipole-to-local translation, and tests only the
// stars of the other cells one by one: the cell expansion of distant stars
// that tree codes rest on, at the same truncation bound per cell.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ray_common.h"

namespace raysh {

namespace {

constexpr int kOrder = 24;            // Taylor terms B_0 .. B_kOrder
constexpr int kWaves = kThreads / 64;
constexpr int kNearPerWave = 512;     // near-star list capacity of each wave
constexpr int kCX = 4, kCY = 4;       // rays per lane
constexpr int kTile = kLanesX * kCX;  // 64 rays per tile side
static_assert(kLanesX * kCX == kLanesY * kCY, "square tiles");

constexpr int kMaxTiles = 16;         // tiles per workgroup block, at most 4 x 4
constexpr int kCellMaxRows = kThreads;   // star-cell grid rows and columns: one thread per row
constexpr int kCellMaxCells = 4096;
constexpr int64_t kCellMaxStars = int64_t(1) << 26;   // the host keeps two copies while building
constexpr int32_t kCellMaxPerCell = 1 << 20;          // stars of one cell (its multipoles take one thread)

struct ExpShared {
    double2 A[kOrder + 1];                      // the block's coefficients
    double2 B[kMaxTiles][kOrder + 1];           // each tile's coefficients (blocks of more than one tile)
    double2 part[kWaves][kOrder + 1];           // per-wave partial sums
    int outer_idx[kWaves][kNearPerWave];        // the block's near stars, each wave's in index order
    int outer_n[kWaves];
    int inner_idx[kWaves][kNearPerWave];        // the tile's near stars (a subset of the block's)
    int inner_n[kWaves];
    int row_lo[kCellMaxRows], row_hi[kCellMaxRows];   // each star-cell row's band of open cells
    int row_first[kCellMaxRows];                      // first record of the band's stars
    int row_pref[kCellMaxRows];                       // the bands' stars before this row
    int wave_tot[kWaves];
};

// What a block's pass over the stars leaves for its tiles: the block's
// coefficients and its near stars, each wave's list in order (the counts
// include stars beyond the lists' capacity).
struct BlockFar {
    double2 A[kOrder + 1];
    int outer_n[kWaves];
    int outer_idx[kWaves][kNearPerWave];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}

// Centre and radius (centre to corner ray, slightly enlarged) of the square
// of w x w lattice points whose first point is (i, j) of the block.
__device__ __forceinline__ void region(const ShootParams &p, int64_t i, int64_t j, int w, double &cx,
                                       double &cy, double &rho) {
    const double x_first = image_angle(p.x0, p.i0 + i, p.dx);
    const double x_last = image_angle(p.x0, p.i0 + i + w - 1, p.dx);
    const double y_first = image_angle(p.y0, p.j0 + j, p.dy);
    const double y_last = image_angle(p.y0, p.j0 + j + w - 1, p.dy);
    cx = 0.5 * (x_first + x_last);
    cy = 0.5 * (y_first + y_last);
    const double hx = 0.5 * (x_last - x_first), hy = 0.5 * (y_last - y_first);
    rho = __builtin_sqrt(hx * hx + hy * hy) * (1.0 + 1e-12) + 1e-290;
}

// region() for a square every lane of the wave shares: the results are
// moved to scalar registers.
__device__ __forceinline__ void region_uniform(const ShootParams &p, int64_t i, int64_t j, int w, double &cx,
                                               double &cy, double &rho) {
    region(p, i, j, w, cx, cy, rho);
    cx = uniform_f64(cx);
    cy = uniform_f64(cy);
    rho = uniform_f64(rho);
}

// One pass over `count` entries split into four contiguous quarters, one per
// wave.  fetch(e, k, x, y, m) gives entry e's star: its index k and record.
// A star farther than sqrt(r_near2) from (cx, cy) adds m u (-u rho)^q to
// the lane's coefficients; a nearer one is appended to its wave's out list,
// so that the concatenated out lists keep the entries' order.  out_n counts
// every near star, also beyond the capacity.
template <class Fetch>
__device__ __forceinline__ void p2l_pass(int count, Fetch fetch, double cx, double cy, double rho, double r_near2,
                                         double2 (&acc)[kOrder + 1], int (*out_idx)[kNearPerWave], int *out_n) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int per_wave = (count + kWaves - 1) / kWaves;
    const int w0 = wave * per_wave < count ? wave * per_wave : count;
    const int w1 = w0 + per_wave < count ? w0 + per_wave : count;
    int found = 0;   // this wave's near stars so far (uniform in the wave)
    for (int base = w0; base < w1; base += 64) {
        const int e = base + lane;
        bool near = false;
        int k = 0;
        if (e < w1) {
            double sx, sy, sm;
            fetch(e, k, sx, sy, sm);
            const double dx = cx - sx, dy = cy - sy;
            const double d2 = dx * dx + dy * dy;
            near = d2 <= r_near2;
            if (!near) {
                const double inv = 1.0 / d2;
                const double2 u = make_double2(dx * inv, -dy * inv);        // 1 / (c - z_k)
                const double2 mu = make_double2(-u.x * rho, -u.y * rho);    // -u rho
                double2 t = make_double2(sm * u.x, sm * u.y);               // m u
#pragma unroll
                for (int q = 0; q <= kOrder; ++q) {
                    acc[q].x += t.x;
                    acc[q].y += t.y;
                    if (q < kOrder) t = cmul(t, mu);
                }
            }
        }
        const unsigned long long ball = __ballot(near);
        if (near) {
            const int pos = found + __popcll(ball & ((1ull << lane) - 1ull));
            if (pos < kNearPerWave) out_idx[wave][pos] = k;
        }
        found += __popcll(ball);
    }
    if (lane == 0) out_n[wave] = found;
}

// Binomial coefficients C(j + q, q) for j, q <= kOrder: exact integers (at
// most C(48, 24) < 2^53) built by Pascal's rule at compile time.
struct CellBinomialTable {
    double c[kOrder + 1][kOrder + 1];
};

constexpr CellBinomialTable make_cell_binomials() {
    CellBinomialTable t{};
    for (int j = 0; j <= kOrder; ++j)
        for (int q = 0; q <= kOrder; ++q)
            t.c[j][q] = (j == 0 || q == 0) ? 1.0 : t.c[j - 1][q] + t.c[j][q - 1];
    return t;
}

__constant__ CellBinomialTable kCellBinomial = make_cell_binomials();

// A star cell's multipole expansion (scaled: M_j = sum_k m_k ((z_k - z_c) / r_c)^j)
// translated to the local expansion of a region of centre C and radius
// rho, added to acc.  With D = C - z_c, w = 1/D and g = -rho w,
//   sum_k m_k / (C + rho s - z_k) = w sum_j M_j (r_c w)^j sum_q C(j + q, q) g^q s^q,
// which converges for (r_c + rho) < |D| and, truncated at kOrder in j and
// q, leaves at most theta^(kOrder+1) / (1 - theta) of the cell's field with
// theta = (r_c + rho) / |D|, the bound of the per-star expansion.
__device__ __forceinline__ void m2l_cell(const double2 *M, double dx, double dy, double rc, double rho,
                                         double2 (&acc)[kOrder + 1]) {
    const double inv = 1.0 / (dx * dx + dy * dy);
    const double2 w = make_double2(dx * inv, -dy * inv);
    const double2 g = make_double2(-rho * w.x, -rho * w.y);
    const double2 a = make_double2(rc * w.x, rc * w.y);
    double2 ap = w;   // w (r_c w)^j
    for (int j = 0; j <= kOrder; ++j) {   // uniform trip count
        double2 t = cmul(M[j], ap);
#pragma unroll
        for (int q = 0; q <= kOrder; ++q) {
            const double b = kCellBinomial.c[j][q];
            acc[q].x = __builtin_fma(b, t.x, acc[q].x);
            acc[q].y = __builtin_fma(b, t.y, acc[q].y);
            if (q < kOrder) t = cmul(t, g);
        }
        ap = cmul(ap, a);
    }
}

// Exclusive prefix sum of one int per thread over the workgroup (values of
// threads past `n` count as zero); returns the thread's prefix and writes the
// total to *total.  Every thread of the workgroup must call it.
__device__ __forceinline__ int block_exclusive_scan(int v, int *wave_tot, int *total) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int up = __shfl_up(incl, off, 64);
        if (lane >= off) incl += up;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) before += wave_tot[w];
        all += wave_tot[w];
    }
    *total = all;
    return before + incl - v;
}

// Workgroup sum of the lanes' coefficients into dst (added to it when ADD),
// in a fixed order.  Within a wave the 2 (kOrder + 1) real components,
// padded with zeros to 64 slots, are reduced by recursive halving: at the
// step of lane mask m, lanes with that bit keep the upper half of their
// slots and the others the lower half, each adds the half its partner
// sends, so after six steps lane l holds the wave's sum of slot l (126
// exchanges per lane instead of 300 for a butterfly over every slot).
// The waves' sums are then added in turn.
template <bool ADD>
__device__ __forceinline__ void reduce_coeffs(double2 (&acc)[kOrder + 1], ExpShared &ex, double2 *dst) {
    constexpr int kSlots = 2 * (kOrder + 1);
    static_assert(kSlots <= 64, "one slot per lane at the end");
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    double v[64];
#pragma unroll
    for (int q = 0; q <= kOrder; ++q) {
        v[2 * q] = acc[q].x;
        v[2 * q + 1] = acc[q].y;
    }
#pragma unroll
    for (int i = kSlots; i < 64; ++i) v[i] = 0.0;
#pragma unroll
    for (int n = 64; n > 1; n /= 2) {
        const int m = n / 2;                 // the lane bit of this step
        const bool upper = (lane & m) != 0;
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            const double keep = upper ? v[i + n / 2] : v[i];
            const double send = upper ? v[i] : v[i + n / 2];
            v[i] = keep + __shfl_xor(send, m, 64);
        }
    }
    double *part = reinterpret_cast<double *>(&ex.part[wave][0]);
    if (lane < kSlots) part[lane] = v[0];
    __syncthreads();
    if (threadIdx.x < kSlots) {
        double t = reinterpret_cast<const double *>(&ex.part[0][0])[threadIdx.x];
        for (int w = 1; w < kWaves; ++w) t += reinterpret_cast<const double *>(&ex.part[w][0])[threadIdx.x];
        double *d = reinterpret_cast<double *>(dst);
        if (ADD) t += d[threadIdx.x];
        d[threadIdx.x] = t;
    }
    __syncthreads();
}

// Binomial coefficients C(n, k) for n, k <= kOrder: exact integers (at most
// C(24, 12)) built by Pascal's rule at compile time.
struct BinomialTable {
    double c[kOrder + 1][kOrder + 1];
};

constexpr BinomialTable make_binomials() {
    BinomialTable t{};
    for (int n = 0; n <= kOrder; ++n) {
        t.c[n][0] = 1.0;
        for (int k = 1; k <= n; ++k) t.c[n][k] = t.c[n - 1][k - 1] + (k < n ? t.c[n - 1][k] : 0.0);
    }
    return t;
}

__constant__ BinomialTable kBinomial = make_binomials();

// Coefficient r of the block's polynomial re-centred on a tile: with
// s = a + b s' (a = (c - C) / R, b = rho / R),
//   B_r = b^r sum_{q=r}^{kOrder} A_q C(q, r) a^(q - r),
// summed by Horner in a from q = kOrder down.
__device__ __forceinline__ double2 shift_coeff(const double2 *A, int r, double2 a, double b) {
    double2 acc = make_double2(A[kOrder].x * kBinomial.c[kOrder][r], A[kOrder].y * kBinomial.c[kOrder][r]);
    for (int q = kOrder - 1; q >= r; --q) {
        const double c = kBinomial.c[q][r];
        const double2 t = cmul(acc, a);
        acc = make_double2(t.x + A[q].x * c, t.y + A[q].y * c);
    }
    double br = 1.0;
    for (int i = 0; i < r; ++i) br *= b;
    return make_double2(acc.x * br, acc.y * br);
}

// The FP64 term of star k for a lane's rays (reciprocal plus one Newton
// step, as in the one-pass kernel).
__device__ __forceinline__ void direct_star(const ConstStar *st, int k, const double (&tx)[kCX],
                                            const double (&ty)[kCY], double (&ax)[kCY][kCX],
                                            double (&ay)[kCY][kCX]) {
    const double sx = st[k].x, sy = st[k].y, sm = st[k].m;
#pragma unroll
    for (int b = 0; b < kCY; ++b) {
        const double ey = ty[b] - sy;
#pragma unroll
        for (int a = 0; a < kCX; ++a) {
            const double ex_ = tx[a] - sx;
            const double r2 = __builtin_fma(ex_, ex_, ey * ey);
            double y = __builtin_amdgcn_rcp(r2);
            const double e = __builtin_fma(-r2, y, 1.0);
            y = __builtin_fma(y, e, y);
            const double wgt = sm * y;
            ax[b][a] = __builtin_fma(wgt, ex_, ax[b][a]);
            ay[b][a] = __builtin_fma(wgt, ey, ay[b][a]);
        }
    }
}

// The block pass over star cells.  A cell whose centre is at least
// (r_c + rho) / theta_open from the block's centre enters the block's
// coefficients through its multipole expansion (m2l_cell); the rest form,
// in each row of the cell grid, a band of open cells whose stars are tested
// one by one as in the pass over every star, so the near lists hold the
// same stars (in cell order, index order within a cell).
__device__ __forceinline__ void block_pass_cells(const StarCells &cells, double bcx, double bcy, double brho,
                                                 double inv_theta, double r_near2, double2 (&acc)[kOrder + 1],
                                                 ExpShared &ex) {
    const int ncx = uniform(cells.ncx), ncy = uniform(cells.ncy);
    const double h = uniform_f64(cells.h), rc = uniform_f64(cells.rc);
    const double gx0 = uniform_f64(cells.gx0), gy0 = uniform_f64(cells.gy0);
    const double rmac = (rc + brho) * inv_theta;
    const double rmac2 = rmac * rmac;
    // row j (one thread each): its band [lo, hi] and the band's stars
    const int j = threadIdx.x;
    int first = 0, cnt = 0;
    if (j < ncy) {
        const double dy = bcy - (gy0 + ((double)j + 0.5) * h);
        int lo = ncx, hi = -1;
        for (int i = 0; i < ncx; ++i) {
            const double dx = bcx - (gx0 + ((double)i + 0.5) * h);
            if (dx * dx + dy * dy < rmac2) {
                if (lo > i) lo = i;
                hi = i;
            }
        }
        ex.row_lo[j] = lo;
        ex.row_hi[j] = hi;
        if (hi >= lo) {
            first = cells.start[j * ncx + lo];
            cnt = cells.start[j * ncx + hi + 1] - first;
        }
        ex.row_first[j] = first;
    }
    int total = 0;
    const int pref = block_exclusive_scan(cnt, ex.wave_tot, &total);   // its barrier publishes the bands
    if (j < ncy) ex.row_pref[j] = pref;
    __syncthreads();
    // every non-empty cell outside the bands, through its multipole expansion
    const int n_cells = ncx * ncy;
    for (int c = threadIdx.x; c < n_cells; c += kThreads) {
        const int i = c % ncx, jj = c / ncx;
        if (i >= ex.row_lo[jj] && i <= ex.row_hi[jj]) continue;
        if (cells.start[c + 1] == cells.start[c]) continue;
        const double dx = bcx - (gx0 + ((double)i + 0.5) * h);
        const double dy = bcy - (gy0 + ((double)jj + 0.5) * h);
        m2l_cell(cells.mult + (size_t)c * (kOrder + 1), dx, dy, rc, brho, acc);
    }
    // the bands' stars, one by one: entry e is in the last row whose prefix
    // is at most e (rows before it hold fewer stars, empty rows share their
    // successor's prefix)
    const Star *sorted = cells.sorted;
    p2l_pass(
        uniform(total),
        [&](int e, int &k, double &x, double &y, double &m) {
            int lo = 0, hi = ncy - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (ex.row_pref[mid] <= e) lo = mid;
                else hi = mid - 1;
            }
            const Star st = sorted[ex.row_first[lo] + (e - ex.row_pref[lo])];
            x = st.x;
            y = st.y;
            m = st.m;
            k = (int)__builtin_bit_cast(long long, st.pad);
        },
        bcx, bcy, brho, r_near2, acc, ex.outer_idx, ex.outer_n);
}

// The block pass, one workgroup per block of block_rays x block_rays rays:
// the stars far from the block enter its local expansion A (through star
// cells when CELLS), the near ones go to its lists; both are written to
// far[blockIdx.x] for the tile kernel.  Two workgroups per compute unit: the
// cells' translations need the registers.
template <bool CELLS>
__global__ __launch_bounds__(kThreads, 2) void expansion_block_kernel(ShootParams p, StarCells cells,
                                                                      double theta_open, int blocks_x,
                                                                      int block_rays, BlockFar *__restrict__ far) {
    __shared__ ExpShared ex;
    const int64_t b_i = (int64_t)(blockIdx.x % blocks_x) * block_rays;
    const int64_t b_j = (int64_t)(blockIdx.x / blocks_x) * block_rays;
    const ConstStar *st = const_stars(uniform_ptr(p.stars));
    const int n = uniform(p.n_stars);
    const double inv_theta = uniform_f64(1.0 / theta_open);
    double bcx, bcy, brho;
    region_uniform(p, b_i, b_j, block_rays, bcx, bcy, brho);
    double2 acc[kOrder + 1];
#pragma unroll
    for (int q = 0; q <= kOrder; ++q) acc[q] = make_double2(0.0, 0.0);
    const double r_near = brho * inv_theta;
    const double r_near2 = uniform_f64(r_near * r_near);
    if constexpr (CELLS) {
        block_pass_cells(cells, bcx, bcy, brho, inv_theta, r_near2, acc, ex);
    } else {
        p2l_pass(
            n,
            [&](int e, int &k, double &x, double &y, double &m) {
                k = e;
                x = st[e].x;
                y = st[e].y;
                m = st[e].m;
            },
            bcx, bcy, brho, r_near2, acc, ex.outer_idx, ex.outer_n);
    }
    reduce_coeffs<false>(acc, ex, ex.A);   // its barriers also publish outer_n
    BlockFar *f = far + blockIdx.x;
    if (threadIdx.x <= kOrder) f->A[threadIdx.x] = ex.A[threadIdx.x];
    if (threadIdx.x < kWaves) f->outer_n[threadIdx.x] = ex.outer_n[threadIdx.x];
    for (int w = 0; w < kWaves; ++w) {
        const int cnt = min(ex.outer_n[w], kNearPerWave);
        for (int i = threadIdx.x; i < cnt; i += kThreads) f->outer_idx[w][i] = ex.outer_idx[w][i];
    }
}

// The tiles of a block of L x L tiles, after its block pass: workgroup g
// takes tiles [TPW s, TPW (s + 1)) of block g / (L^2 / TPW), s = g mod
// (L^2 / TPW).  WPS waves per SIMD (workgroups per compute unit).
template <int L, int TPW, int WPS>
__global__ __launch_bounds__(kThreads, WPS) void expansion_fp64_kernel(ShootParams p, double theta_open,
                                                                       int blocks_x,
                                                                       const BlockFar *__restrict__ far) {
    static_assert(TPW >= 1 && (L * L) % TPW == 0, "whole groups of a block's tiles");
    constexpr int kSubs = L * L / TPW;
    __shared__ BinShared sh;
    __shared__ ExpShared ex;
    bin_shared_init(sh);
    for (int t = threadIdx.x; t < kWinX * kWinY; t += kThreads) sh.win[t] = 0;   // kept clear by finish_tile

    const int lx = threadIdx.x % kLanesX;
    const int ly = threadIdx.x / kLanesX;
    const int blk = (int)(blockIdx.x / kSubs);
    const int t_begin = (int)(blockIdx.x % kSubs) * TPW, t_end = t_begin + TPW;
    const int64_t b_i = (int64_t)(blk % blocks_x) * (kTile * L);
    const int64_t b_j = (int64_t)(blk / blocks_x) * (kTile * L);
    const ConstStar *st = const_stars(uniform_ptr(p.stars));
    const int n = uniform(p.n_stars);
    const double inv_theta = uniform_f64(1.0 / theta_open);

    // --- the block: its coefficients A and near stars, from the block pass
    double bcx, bcy, brho;
    region_uniform(p, b_i, b_j, kTile * L, bcx, bcy, brho);
    {
        const BlockFar *f = far + blk;
        if (threadIdx.x <= kOrder) ex.A[threadIdx.x] = f->A[threadIdx.x];
        if (threadIdx.x < kWaves) ex.outer_n[threadIdx.x] = f->outer_n[threadIdx.x];
        for (int w = 0; w < kWaves; ++w) {
            const int cnt = min(uniform(f->outer_n[w]), kNearPerWave);
            for (int i = threadIdx.x; i < cnt; i += kThreads) ex.outer_idx[w][i] = f->outer_idx[w][i];
        }
        __syncthreads();
    }
    bool overflow = false;
    int n_outer = 0;
    for (int w = 0; w < kWaves; ++w) {
        overflow |= ex.outer_n[w] > kNearPerWave;
        n_outer += ex.outer_n[w];
    }
    if (L > 1 && !overflow) {   // uniform
        // the block's polynomial re-centred on every tile of the workgroup at once
        const double inv_brho = 1.0 / brho;
        for (int idx = threadIdx.x; idx < TPW * (kOrder + 1); idx += kThreads) {
            const int t = t_begin + idx / (kOrder + 1), r = idx % (kOrder + 1);
            double cx, cy, rho;
            region(p, b_i + (int64_t)(t % L) * kTile, b_j + (int64_t)(t / L) * kTile, kTile, cx, cy, rho);
            ex.B[t][r] = shift_coeff(ex.A, r, make_double2((cx - bcx) * inv_brho, (cy - bcy) * inv_brho),
                                     rho * inv_brho);
        }
        __syncthreads();
    }

    for (int t = t_begin; t < t_end; ++t) {   // uniform trip count
        const int64_t tile_i = b_i + (int64_t)(t % L) * kTile;
        const int64_t tile_j = b_j + (int64_t)(t / L) * kTile;
        if (tile_i >= p.nx || tile_j >= p.ny) continue;   // uniform: no ray of this tile is in the lattice block

        const int(*near_idx)[kNearPerWave] = ex.outer_idx;
        const int *near_n = ex.outer_n;
        const double2 *coef = ex.B[L == 1 ? 0 : t];
        double cx = bcx, cy = bcy, rho = brho;
        if (L == 1 && !overflow) {   // uniform
            // a copy per tile: read from a buffer the loop writes, the
            // coefficients stay in LDS instead of 100 VGPRs
            if (threadIdx.x <= kOrder) ex.B[0][threadIdx.x] = ex.A[threadIdx.x];
            __syncthreads();
        }
        if (L > 1 && !overflow) {   // uniform
            region_uniform(p, tile_i, tile_j, kTile, cx, cy, rho);
            double2 acc[kOrder + 1];
#pragma unroll
            for (int q = 0; q <= kOrder; ++q) acc[q] = make_double2(0.0, 0.0);
            const double r_near = rho * inv_theta;
            const int n0 = ex.outer_n[0], n1 = n0 + ex.outer_n[1], n2 = n1 + ex.outer_n[2];
            p2l_pass(
                uniform(n_outer),
                [&](int e, int &k, double &x, double &y, double &m) {
                    k = e < n0   ? ex.outer_idx[0][e]
                        : e < n1 ? ex.outer_idx[1][e - n0]
                        : e < n2 ? ex.outer_idx[2][e - n1]
                                 : ex.outer_idx[3][e - n2];
                    x = st[k].x;
                    y = st[k].y;
                    m = st[k].m;
                },
                cx, cy, rho, uniform_f64(r_near * r_near), acc, ex.inner_idx, ex.inner_n);
            reduce_coeffs<true>(acc, ex, ex.B[t]);   // its barriers also publish inner_n
            near_idx = ex.inner_idx;
            near_n = ex.inner_n;
        }

        double tx[kCX], ty[kCY];
#pragma unroll
        for (int a = 0; a < kCX; ++a) tx[a] = image_angle(p.x0, p.i0 + tile_i + lx + kLanesX * a, p.dx);
#pragma unroll
        for (int b = 0; b < kCY; ++b) ty[b] = image_angle(p.y0, p.j0 + tile_j + ly + kLanesY * b, p.dy);
        double ax[kCY][kCX], ay[kCY][kCX];
        if (!overflow) {
            // far field: Horner in s = (z - c) / rho for the lane's rays
            // together, one coefficient at a time (one LDS read each);
            // f = alpha_x - i alpha_y is then added to the macro term
            const double inv_rho = 1.0 / rho;
            double wx[kCX], wy[kCY];
#pragma unroll
            for (int a = 0; a < kCX; ++a) wx[a] = (tx[a] - cx) * inv_rho;
#pragma unroll
            for (int b = 0; b < kCY; ++b) wy[b] = (ty[b] - cy) * inv_rho;
            const double2 top = coef[kOrder];
#pragma unroll
            for (int b = 0; b < kCY; ++b)
#pragma unroll
                for (int a = 0; a < kCX; ++a) {
                    ax[b][a] = top.x;
                    ay[b][a] = top.y;
                }
            for (int q = kOrder - 1; q >= 0; --q) {
                const double2 bq = coef[q];
#pragma unroll
                for (int b = 0; b < kCY; ++b)
#pragma unroll
                    for (int a = 0; a < kCX; ++a) {
                        const double fx = ax[b][a], fy = ay[b][a];
                        ax[b][a] = __builtin_fma(fx, wx[a], __builtin_fma(-fy, wy[b], bq.x));
                        ay[b][a] = __builtin_fma(fx, wy[b], __builtin_fma(fy, wx[a], bq.y));
                    }
            }
#pragma unroll
            for (int b = 0; b < kCY; ++b)
#pragma unroll
                for (int a = 0; a < kCX; ++a) {
                    double mx, my;
                    macro_term(p, tx[a], ty[b], mx, my);
                    ax[b][a] = mx + ax[b][a];
                    ay[b][a] = my - ay[b][a];
                }
            // near stars, directly, in index order
            for (int w = 0; w < kWaves; ++w) {
                const int cnt = uniform(near_n[w]);
                for (int i = 0; i < cnt; ++i) direct_star(st, uniform(near_idx[w][i]), tx, ty, ax, ay);
            }
        } else {
            // too many near stars for the lists: every star directly
#pragma unroll
            for (int b = 0; b < kCY; ++b)
#pragma unroll
                for (int a = 0; a < kCX; ++a) macro_term(p, tx[a], ty[b], ax[b][a], ay[b][a]);
            for (int k = 0; k < n; ++k) direct_star(st, k, tx, ty, ax, ay);
        }
        finish_tile<kCX, kCY, kWinX, kWinY, true>(p, sh, tx, ty, ax, ay, tile_i, tile_j, lx, ly);
        __syncthreads();   // the bin window, red[], B and the inner lists are reused by the next tile
        bin_shared_init(sh);
    }
}

// The block pass (with or without cells), then the tiles at three
// workgroups per compute unit (measured faster than two at every star count
// once the block pass is a kernel of its own), one row of a block's tiles
// per workgroup: L times as many workgroups as blocks, so that the last
// round of a launch is a small part of it (on the 8192^2 lattice of 16384
// stars, 1024 workgroups of 16 tiles filled 1.33 rounds of 768; 4096 of 4
// tiles run 11 % faster, and rows beat 2, 8 or 16 tiles per workgroup).
template <int L>
hipError_t launch_level(const ShootParams &p, const StarCells &cells, double theta_open, int64_t tiles_x,
                        int64_t tiles_y, BlockFar *far, hipStream_t s) {
    const int64_t bx = (tiles_x + L - 1) / L, by = (tiles_y + L - 1) / L;
    const dim3 grid((unsigned)(bx * by));
    if (cells.ncx > 0)
        hipLaunchKernelGGL(expansion_block_kernel<true>, grid, dim3(kThreads), 0, s, p, cells, theta_open, (int)bx,
                           kTile * L, far);
    else
        hipLaunchKernelGGL(expansion_block_kernel<false>, grid, dim3(kThreads), 0, s, p, cells, theta_open, (int)bx,
                           kTile * L, far);
    hipLaunchKernelGGL((expansion_fp64_kernel<L, L, 3>), dim3((unsigned)(bx * by * L)), dim3(kThreads), 0, s, p,
                       theta_open, (int)bx, far);
    return hipGetLastError();
}

// Each star cell's scaled multipole expansion, one thread per cell, its
// stars in their sorted order.
__global__ __launch_bounds__(kThreads) void star_cell_multipole_kernel(const Star *__restrict__ sorted,
                                                                      const int32_t *__restrict__ start, int ncx,
                                                                      int ncy, double gx0, double gy0, double h,
                                                                      double rc, double2 *__restrict__ mult) {
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= ncx * ncy) return;
    const double cx = gx0 + ((double)(c % ncx) + 0.5) * h;
    const double cy = gy0 + ((double)(c / ncx) + 0.5) * h;
    const double inv = 1.0 / rc;
    double2 acc[kOrder + 1];
#pragma unroll
    for (int q = 0; q <= kOrder; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int i = start[c]; i < start[c + 1]; ++i) {
        const Star st = sorted[i];
        const double2 t = make_double2((st.x - cx) * inv, (st.y - cy) * inv);   // (z_k - z_c) / r_c
        double2 tp = make_double2(st.m, 0.0);
#pragma unroll
        for (int q = 0; q <= kOrder; ++q) {
            acc[q].x += tp.x;
            acc[q].y += tp.y;
            if (q < kOrder) tp = cmul(tp, t);
        }
    }
#pragma unroll
    for (int q = 0; q <= kOrder; ++q) mult[(size_t)c * (kOrder + 1) + q] = acc[q];
}

}  // namespace

int expansion_order() { return kOrder; }

// The block that minimises a simple cost model fitted on MI355X: a block
// costs about N* + 16384 L^2 star-equivalents (its pass over all stars,
// then L^2 tiles of Horner steps, near stars and binning), and blocks run in
// rounds of three per compute unit, a part-filled round counted in
// proportion.  The tiles of a block run as L workgroups, but the model
// keeps their sum: it also keeps large blocks away from lattices of few
// blocks, where dense star fields would overflow a large block's near-star
// lists (then its tiles sum every star directly).  Counting the tile
// workgroups as separate work picked 4 x 4 blocks for the 4096^2-ray maps
// of 512 to 50 000 stars, five times slower than 2 x 2.
int expansion_block(int64_t nx, int64_t ny, int64_t n_stars, int n_cu) {
    const int64_t tx = (nx + kTile - 1) / kTile, ty = (ny + kTile - 1) / kTile;
    const int64_t slots = 3 * (int64_t)(n_cu > 0 ? n_cu : 256);
    int best = 1;
    double best_cost = 0.0;
    for (int L : {1, 2, 4}) {
        const int64_t blocks = ((tx + L - 1) / L) * ((ty + L - 1) / L);
        const double rounds = std::max(1.0, (double)blocks / (double)slots);   // a part-filled round runs faster
        const double cost = rounds * ((double)n_stars + 16384.0 * L * L);
        if (L == 1 || cost < best_cost) {
            best = L;
            best_cost = cost;
        }
    }
    return best;
}

size_t expansion_workspace_bytes(int64_t nx, int64_t ny, int block) {
    const int64_t tiles_x = (nx + kTile - 1) / kTile, tiles_y = (ny + kTile - 1) / kTile;
    const int64_t blocks = ((tiles_x + block - 1) / block) * ((tiles_y + block - 1) / block);
    return (size_t)blocks * sizeof(BlockFar);
}

hipError_t launch_shoot_expansion(const ShootParams &p, const StarCells &cells, double theta_open, int block,
                                  void *workspace, hipStream_t s) {
    ShootParams q = p;
    const int64_t tiles_x = (p.nx + kTile - 1) / kTile;
    const int64_t tiles_y = (p.ny + kTile - 1) / kTile;
    q.tiles_x = (int32_t)tiles_x;
    BlockFar *far = static_cast<BlockFar *>(workspace);
    switch (block) {
        case 1: return launch_level<1>(q, cells, theta_open, tiles_x, tiles_y, far, s);
        case 2: return launch_level<2>(q, cells, theta_open, tiles_x, tiles_y, far, s);
        case 4: return launch_level<4>(q, cells, theta_open, tiles_x, tiles_y, far, s);
        default: return hipErrorInvalidValue;
    }
}

void free_star_cells(StarCellStore &c) {
    if (c.sorted) (void)hipFree(c.sorted);
    if (c.start) (void)hipFree(c.start);
    if (c.mult) (void)hipFree(c.mult);
    c = StarCellStore{};
}

// The cell side balances a block's two costs: the stars of its open cells,
// tested one by one (their number grows as side^2), against the
// translations of the other cells (whose number falls as 1/side^2, each
// about 26 times the work of one star's expansion).  Their sum is least
// near side = sqrt(area / sqrt(N*)) for theta_open = 0.25; the grid is then
// coarsened until it fits the workgroup's tables.
hipError_t build_star_cells(const Star *d_stars, int64_t n_stars, hipStream_t s, StarCellStore &out) {
    free_star_cells(out);
    if (n_stars < 2 || n_stars > kCellMaxStars) return hipSuccess;   // no cells
    std::vector<Star> host((size_t)n_stars);
    hipError_t e = hipMemcpyAsync(host.data(), d_stars, (size_t)n_stars * sizeof(Star), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    double x0 = host[0].x, x1 = host[0].x, y0 = host[0].y, y1 = host[0].y;
    for (const Star &st : host) {
        x0 = std::min(x0, st.x);
        x1 = std::max(x1, st.x);
        y0 = std::min(y0, st.y);
        y1 = std::max(y1, st.y);
    }
    const double w = x1 - x0, hgt = y1 - y0, big = std::max(w, hgt);
    if (!(big > 0.0)) return hipSuccess;   // every star at one point: no cells
    const double area = std::max(w * hgt, 1e-6 * big * big);
    double side = std::sqrt(area / std::sqrt((double)n_stars));
    int ncx = 0, ncy = 0;
    for (;;) {
        ncx = (int)std::min(std::floor(w / side) + 1.0, 1e9);
        ncy = (int)std::min(std::floor(hgt / side) + 1.0, 1e9);
        if (ncx <= kCellMaxRows && ncy <= kCellMaxRows && (int64_t)ncx * ncy <= kCellMaxCells) break;
        side *= 1.25;
    }
    const int n_cells = ncx * ncy;
    // counting sort of the stars by cell, index order within a cell
    std::vector<int32_t> cell((size_t)n_stars), start((size_t)n_cells + 1, 0);
    for (int64_t k = 0; k < n_stars; ++k) {
        const int i = std::min((int)((host[k].x - x0) / side), ncx - 1);
        const int j = std::min((int)((host[k].y - y0) / side), ncy - 1);
        cell[k] = j * ncx + i;
        ++start[cell[k] + 1];
    }
    int32_t most = 0;
    for (int c = 0; c < n_cells; ++c) most = std::max(most, start[c + 1]);
    if (most > kCellMaxPerCell) return hipSuccess;   // one thread per cell would take too long: no cells
    for (int c = 0; c < n_cells; ++c) start[c + 1] += start[c];
    std::vector<Star> sorted((size_t)n_stars);
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t k = 0; k < n_stars; ++k) {
            Star st = host[k];
            st.pad = __builtin_bit_cast(double, (long long)k);   // the star's index
            sorted[fill[cell[k]]++] = st;
        }
    }
    StarCellStore c;
    e = hipMalloc(&c.sorted, (size_t)n_stars * sizeof(Star));
    if (e == hipSuccess) e = hipMalloc(&c.start, ((size_t)n_cells + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&c.mult, (size_t)n_cells * (kOrder + 1) * sizeof(double2));
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.sorted, sorted.data(), (size_t)n_stars * sizeof(Star), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.start, start.data(), ((size_t)n_cells + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                           s);
    // cells hold every star in the closed square of their cell (the last row
    // and column also the stars on the far edge): r_c is the half-diagonal,
    // enlarged for the rounding of the cell assignment
    const double rc = side * std::sqrt(0.5) * (1.0 + 1e-12);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(star_cell_multipole_kernel, dim3((unsigned)((n_cells + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, s, c.sorted, c.start, ncx, ncy, x0, y0, side, rc, c.mult);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host tables are released on return
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_star_cells(c);
        return e;
    }
    c.view = StarCells{c.sorted, c.start, c.mult, x0, y0, side, rc, ncx, ncy};
    out = c;
    return hipSuccess;
}

}  // namespace raysh
