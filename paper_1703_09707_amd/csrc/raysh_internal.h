// Internal declarations shared by the raysh HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raysh.h"

namespace raysh {

// One star as the kernels read it: FP64 position, mass and a pad word so
// that a record is 32 bytes (one scalar 8-dword load).
struct Star {
    double x, y, m, pad;
};

// Everything a shooting kernel needs for one (lens, ray block, window).
// Passed by value: it lands in the kernel-argument segment and is read with
// scalar loads.
struct ShootParams {
    // Eq. (3), first term: K = [[k11, k12], [k12, k22]]
    double k11, k12, k22;
    const Star *stars;
    int32_t n_stars;
    int32_t tiles_x;           // ray tiles per lattice row of this block
    // ray lattice block
    double x0, y0, dx, dy;
    int64_t nx, ny, i0, j0;
    // source window
    double X0, Y0, Px, Py;
    int32_t NX, NY;
    // outputs (any may be null)
    double *beta_x, *beta_y;
    int32_t *bin;
    int32_t *counts;
    unsigned long long *n_binned;
};

// One parameter set of a batch: its shooting parameters and the range of
// work items (ray tiles) it owns in the batch's queue order.
struct BatchSet {
    ShootParams p;
    int64_t first_item;
    int64_t n_items;
    int64_t n_tiles;          // ray tiles of the set
    int32_t tiles_per_item;   // consecutive tiles one item covers
};

// Arguments of the persistent batch kernels.  Sets are ordered by
// decreasing cost per tile (longest first), items numbered set after set.
struct BatchArgs {
    const BatchSet *sets;
    int32_t n_sets;
    int64_t total_items;
    unsigned long long *queue;   // next item to hand out; zero before launch
};

// Launch shapes selectable per call (the autotuner's search space).
struct TileShape {
    int cx, cy;      // rays per lane along x and y
    int share;       // r^2 values sharing one reciprocal (FP64 path)
    int star_tile;   // FP64: consecutive stars among them (the rest are the lane's
                     // neighbouring rays); FP32-bulk: stars staged in LDS per pass
};

// Launchers (shoot_fp64.hip, shoot_fp32.hip).  Return hipSuccess or the
// launch error; `shape` must be one the launcher supports.
hipError_t launch_shoot_fp64(const ShootParams &p, const TileShape &shape, hipStream_t s);
hipError_t launch_shoot_fp32(const ShootParams &p, const TileShape &shape, hipStream_t s);
bool fp64_shape_supported(const TileShape &shape);
// Compiled shapes: writes up to cap of them, returns how many exist.
int fp64_shape_list(TileShape *out, int cap);
int fp32_shape_list(TileShape *out, int cap);
bool fp32_shape_supported(const TileShape &shape);
int tile_width(const TileShape &shape);   // rays per tile along x (16 * cx)
int tile_height(const TileShape &shape);  // rays per tile along y (16 * cy)

hipError_t launch_batch_fp64(const BatchArgs &b, const TileShape &shape, int blocks, hipStream_t s);
// Split-K FP64: partial star sums over `parts` star ranges into `partial`
// (parts * nx * ny FP64 pairs), then the finishing pass.
hipError_t launch_split_fp64(const ShootParams &p, const TileShape &shape, int parts, double2 *partial,
                             hipStream_t s);
hipError_t launch_batch_fp32(const BatchArgs &b, const TileShape &shape, int blocks, hipStream_t s);
int batch_fp64_blocks_per_cu(const TileShape &shape);
int batch_fp32_blocks_per_cu(const TileShape &shape);
// Workgroups of the one-shot kernels resident per compute unit.
int shoot_fp64_blocks_per_cu(const TileShape &shape);
int shoot_fp32_blocks_per_cu(const TileShape &shape);

// Cells of the star field for the expansion mode: the star records sorted
// by the cell of a regular grid (origin gx0, gy0, side h; cell c = j ncx + i),
// with each cell's scaled multipole expansion.  ncx = 0: no cells.
struct StarCells {
    const Star *sorted;        // star records by cell; pad holds the star's index (int64 bits)
    const int32_t *start;      // [ncx * ncy + 1]: first record of each cell
    const double2 *mult;       // [ncx * ncy][expansion_order() + 1]
    double gx0, gy0, h, rc;    // rc: radius around a cell's centre that holds its stars
    int32_t ncx, ncy;
};

// Device buffers behind a StarCells view (owned by a context).
struct StarCellStore {
    StarCells view{};
    Star *sorted = nullptr;
    int32_t *start = nullptr;
    double2 *mult = nullptr;
};

// Builds the cells of n_stars device star records (host sort, device
// multipoles; synchronous on s).  Leaves out.view.ncx = 0 when cells do not
// apply (fewer than 2 stars, all at one point, or more than the host build
// takes).  Returns the first HIP error.
hipError_t build_star_cells(const Star *d_stars, int64_t n_stars, hipStream_t s, StarCellStore &out);
void free_star_cells(StarCellStore &cells);

// FP64 with the far field as local expansions (shoot_expansion.hip); tiles
// of 64 x 64 rays in blocks of `block` x `block` tiles (1, 2 or 4): one
// workgroup per block for the pass over the stars, one per row of a block's
// tiles for the tiles.  expansion_block picks the block for a lattice block.  With
// cells (cells.ncx > 0) the block pass takes distant cells through their
// multipole expansions.
hipError_t launch_shoot_expansion(const ShootParams &p, const StarCells &cells, double theta_open, int block,
                                  void *workspace, hipStream_t s);
// Device workspace launch_shoot_expansion needs for an nx x ny lattice block
// (each workgroup block's coefficients and near-star lists, about 8.6 KB each).
size_t expansion_workspace_bytes(int64_t nx, int64_t ny, int block);
int expansion_block(int64_t nx, int64_t ny, int64_t n_stars, int n_cu);
int expansion_order();

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);

}  // namespace raysh
