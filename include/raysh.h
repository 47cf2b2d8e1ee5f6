/*
 * raysh: backward ray shooting through a random star field on AMD MI355X.
 *
 * The method is that of Chen, Kantowski, Dai, Baron & Van der Mark (2017),
 * "Accelerating gravitational microlensing simulations using the Xeon Phi
 * coprocessor" (arXiv:1703.09707):
 *   - the lens equation, Sec. 1, Eq. (1)-(3): a ray at image angle theta
 *     reaches the source plane at beta = theta - alpha with
 *       alpha = K theta + sum_k m_k (theta - theta_k) / |theta - theta_k|^2,
 *       K = [[kappa_c + gamma1, gamma2], [gamma2, kappa_c - gamma1]];
 *     angles are in units of the Einstein angle of the mass unit and m_k in
 *     that mass unit (Eq. (4) and the text after it);
 *   - Algorithm 1 (Sec. 2.2): for every ray of a regular lattice, evaluate
 *     theta, add the macro term and every star's term in index order, form
 *     beta, convert it to a source-plane pixel and, if it lies inside the
 *     source window, add one to that pixel's count (the magnification map).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - Ray (i, j) of a call has global lattice indices (i0 + i, j0 + j) and
 *     image angle theta = (x0 + ((double)(i0+i) + 0.5) * dx,
 *                          y0 + ((double)(j0+j) + 0.5) * dy),
 *     each operation rounded separately, so a block of a lattice reproduces
 *     the rays of the whole lattice bit for bit.
 *   - Pixel (is, js) covers [x0 + is*px, x0 + (is+1)*px) x [y0 + js*py, ...).
 *     The pixel coordinate is (beta - x0) / px with IEEE division, tested
 *     against the window in FP64 before conversion; maps are row-major int32
 *     [ny][nx] with element js*nx + is (the paper's mag[j_s, i_s]).
 *   - A ray whose beta is not finite (it sits exactly on a star) is dropped.
 *
 * Memory: star arrays passed to raysh_init are host memory and are copied;
 * every other pointer (maps, per-ray outputs) is caller-owned DEVICE memory
 * on the context's device.  The library never allocates caller outputs.
 * Work is enqueued on the context's HIP stream and is asynchronous unless a
 * function says otherwise.  Context-owned work buffers (the split-K partial
 * sums, the expansion mode's per-block records, its star cells) are
 * allocated on first use and grown when a larger call needs them; such a
 * call first synchronizes the context's stream, and the first call that
 * uses star cells also copies the stars to the host to build them.
 *
 * Errors: every function returns RAYSH_OK (0) or a RAYSH_E* code, and
 * raysh_last_error() gives a message for the calling thread's last error.
 * Arguments are validated before anything is enqueued: on error nothing is
 * written.  A context is used by one host thread at a time.
 */
#ifndef RAYSH_H
#define RAYSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RAYSH_OK = 0,
    RAYSH_EINVAL = 1,    /* bad argument: NULL, non-finite, non-positive size, unknown precision */
    RAYSH_EOVERFLOW = 2, /* a count or index would not fit the library's integer types */
    RAYSH_ENOMEM = 3,    /* device allocation failed */
    RAYSH_EDEVICE = 4    /* HIP runtime error (including an earlier asynchronous one) */
};

/* Arithmetic of the star sum. */
enum {
    RAYSH_FP64 = 0,          /* every step in FP64 */
    RAYSH_FP32_BULK = 1,     /* star terms in FP32 on tile-relative coordinates,
                                flushed into FP64 sums; theta, the macro term and
                                the beta -> pixel step stay FP64 */
    RAYSH_FP64_EXPANSION = 2 /* FP64; the stars far from a region of rays (farther
                                than rho / theta_open from its centre, rho its
                                radius) enter through one local Taylor expansion
                                of their summed term (order
                                raysh_expansion_order()), the others directly.
                                Regions are blocks of 64 x 64 ray tiles, whose
                                expansion is re-centred on each tile, and the
                                tiles themselves, which re-test only the block's
                                near stars (raysh_set_expansion_block).
                                Truncation error below theta_open^(order+1) *
                                (1 + theta_open) / (1 - theta_open) of each far
                                star's m_k / |theta - theta_k| (1.5e-15 at the
                                default theta_open = 0.25, 1.6e-13 at the
                                largest allowed, 0.3).  The paper names tree
                                codes as the way to avoid the brute-force sum
                                (Sec. 1); this is a two-level form on the ray
                                side. */
};

/* The lens of Eq. (1): smooth convergence, external shear and the stars.
 * x, y, m are HOST arrays of n_stars FP64 values (positions in Einstein
 * angles, masses in the mass unit); they may be NULL when n_stars == 0. */
typedef struct raysh_lens {
    double kappa_c;
    double gamma1;
    double gamma2;
    int64_t n_stars;
    const double *x;
    const double *y;
    const double *m;
} raysh_lens;

/* A block of the image-plane ray lattice (see the theta convention above). */
typedef struct raysh_rays {
    double x0, y0;   /* lattice origin (corner of cell (0, 0)) */
    double dx, dy;   /* lattice spacing, > 0 */
    int64_t nx, ny;  /* rays in this block, >= 0 */
    int64_t i0, j0;  /* global index of the block's first ray, >= 0 */
} raysh_rays;

/* The source window and its pixels (see the pixel convention above). */
typedef struct raysh_pixels {
    double x0, y0;   /* lower-left corner of the window */
    double px, py;   /* pixel size, > 0 */
    int32_t nx, ny;  /* pixels per row and rows, > 0 */
} raysh_pixels;

typedef struct raysh_ctx raysh_ctx;

/*
 * raysh_init: create a context on HIP device `device` whose work goes to
 * HIP stream `hip_stream` (NULL = the null stream), validate the lens and
 * copy the star field to the device (Sec. 2.2: the star field is generated
 * on the host and copied to the accelerator once).
 *   EINVAL: out == NULL; kappa_c or gamma not finite; n_stars < 0; a star
 *           array NULL with n_stars > 0; a position not finite; a mass
 *           negative or not finite.  EOVERFLOW: n_stars > 2^31 - 1.
 *   ENOMEM / EDEVICE from the runtime.  On error *out is left unchanged.
 * The caller may free its star arrays as soon as the call returns.
 */
int raysh_init(raysh_ctx **out, const raysh_lens *lens, int device, void *hip_stream);

/*
 * raysh_set_lens: give an existing context another lens (kappa_c, gamma and
 * star field), as raysh_init would, without creating a context: for runs of
 * many maps of different lenses (the grids of simulations of Sec. 1 and
 * Sec. 2.2).  Waits for all work on the context's device (work enqueued
 * before the call may read the old stars, also in a batch led by another
 * context on another stream), then copies the new stars into its device
 * buffer, growing it when the field is larger (by half again at least),
 * and returns when they are on the device; the caller may then free its
 * arrays.  Captured batch launches that include the context and its star
 * cells are dropped (built again when next used); launch shapes and
 * workspaces are kept.  The context keeps the pinned staging buffers of its
 * uploads (2 x min(N*, 2^19) records of 32 bytes) until raysh_free.
 * Errors as raysh_init (EINVAL also for ctx == NULL); on EINVAL or ENOMEM
 * the context keeps its old lens; after EDEVICE its lens is undefined.
 */
int raysh_set_lens(raysh_ctx *ctx, const raysh_lens *lens);

/* Redirect the context's work to another HIP stream of the same device. */
int raysh_set_stream(raysh_ctx *ctx, void *hip_stream);

/* Number of stars held by the context (0 for a NULL context). */
int64_t raysh_n_stars(const raysh_ctx *ctx);

/*
 * Launch shape of the context's kernels for RAYSH_FP64 or RAYSH_FP32_BULK
 * (the autotuner's knob; results do not depend on it beyond rounding for
 * RAYSH_FP64).  RAYSH_FP64_EXPANSION has one fixed shape; these calls, the
 * tuner and raysh_map_batch return EINVAL for it.  Each lane of a
 * 256-lane workgroup owns cx x cy rays of a (16 cx) x (16 cy) ray tile.
 * RAYSH_FP64: `share` values of r^2 share one reciprocal (a product tree,
 * refined by a Newton step); `star_tile` of them (1, 2 or 4) are consecutive
 * stars of one ray, the rest neighbouring rays of the lane (star_tile 0 in
 * raysh_set_tile means min(share, 4)).  RAYSH_FP32_BULK: `star_tile` stars
 * are staged in LDS per pass (the FP32 partial sums are flushed into FP64
 * after each pass), and `share` must be 0.  EINVAL if the shape is not
 * compiled into the library.
 */
int raysh_set_tile(raysh_ctx *ctx, int precision, int cx, int cy, int share, int star_tile);

/* Far-star criterion of RAYSH_FP64_EXPANSION for this context: a star is
 * expanded when farther than rho / theta_open from the tile centre.  EINVAL
 * outside (0, 0.3], the range in which the truncation error stays below
 * 1e-12 of the error scale S. */
int raysh_set_expansion(raysh_ctx *ctx, double theta_open);

/* Workgroup shape of RAYSH_FP64_EXPANSION for this context: each workgroup
 * expands the stars far from a block of block x block tiles of 64 x 64 rays
 * once, then re-tests only that block's near stars for each tile (block 1:
 * one tile, one test).  0 (the default) picks the block by a cost model:
 * a workgroup costs about n_stars + 16384 block^2 star-equivalents, and
 * workgroups run in rounds of three per compute unit, a part-filled round
 * counted in proportion.  The block
 * changes the order of floating-point operations, not the accuracy bound.
 * EINVAL for a NULL context or a block other than 0, 1, 2 or 4. */
int raysh_set_expansion_block(raysh_ctx *ctx, int block);

/* Star cells of RAYSH_FP64_EXPANSION's block pass.  With cells, the stars
 * are sorted once (per context, on the first call that uses them) by the
 * cell of a regular grid over their bounding box, and each cell gets a
 * multipole expansion of its stars (order raysh_expansion_order(), scaled by
 * the cell's radius r_c).  A cell whose centre lies at least
 * (r_c + rho) / theta_open from a block's centre enters the block's local
 * expansion through it (a multipole-to-local translation: exact algebra
 * up to truncation at the same order and the same error bound per cell);
 * the stars of the other cells are tested one by one as without cells.
 * This is the cell expansion of distant stars that the tree codes of the
 * paper's Sec. 1 rest on.  The near stars are the same with or without
 * cells; their direct sums then go in cell order (index order within a
 * cell) instead of index order.
 *   RAYSH_CELLS_AUTO (default): cells from 65536 stars on (below that the
 *     block pass is a small share of the time, and the build, a round trip
 *     through the host per context, would not pay back within a few maps).
 *   RAYSH_CELLS_ALWAYS: cells whenever the stars span a nonzero box.
 *   RAYSH_CELLS_NEVER: the block pass expands every far star on its own.
 * The grid has at most 4096 cells and 256 rows and columns; building it
 * copies the stars to the host (two copies; at most 2^26 stars, beyond
 * which no cells are used).  EINVAL for a NULL context or another mode. */
enum { RAYSH_CELLS_AUTO = 0, RAYSH_CELLS_ALWAYS = 1, RAYSH_CELLS_NEVER = 2 };
int raysh_set_expansion_cells(raysh_ctx *ctx, int mode);

/* Number of Taylor terms minus one (the order) of RAYSH_FP64_EXPANSION. */
int raysh_expansion_order(void);

/*
 * raysh_set_star_split: split each ray's FP64 star sum over `parts`
 * contiguous star ranges computed by separate workgroups (for many stars
 * and few rays, where one pass over all stars per ray cannot fill the GPU;
 * Sec. 4 of the paper suggests splitting the bending-angle sum between
 * threads).  The partial sums (FP64, one pair per ray and part, in a
 * context-owned workspace of parts * nx * ny * 16 bytes that grows on
 * demand) are added in part order after the macro term; results differ
 * from one pass only by rounding.  parts = 1 (the default) is one pass;
 * parts = 0 picks a count per call from the number of ray tiles and stars
 * (at least 64 stars per part, workspace at most 2 GiB).  Applies to
 * RAYSH_FP64 calls of raysh_shoot and raysh_map.  EINVAL outside [0, 65536];
 * ENOMEM at call time if the workspace cannot be allocated.
 */
int raysh_set_star_split(raysh_ctx *ctx, int parts);

/* The launch shapes compiled for `precision`: writes up to `cap` shapes as
 * 4 ints each (cx, cy, share, star_tile) into `shapes` (may be NULL when
 * cap is 0) and returns how many exist, or -RAYSH_EINVAL for an unknown
 * precision or a negative cap. */
int raysh_list_tiles(int precision, int32_t *shapes, int cap);
int raysh_get_tile(const raysh_ctx *ctx, int precision, int *cx, int *cy, int *share,
                   int *star_tile);

/*
 * raysh_autotune: time every launch shape compiled for `precision` on a
 * sample of the ray block mapped into a scratch map (one warm-up, then the
 * median of three launches), keep the one with the shortest predicted time
 * for the whole block in the context (as raysh_set_tile would) and return it
 * through the optional out-pointers.  A shape's sample is a central part of
 * the block made of whole tiles, in whole rounds of the workgroups the
 * device holds at once (until about 1e11 ray-star interactions or the
 * block's own rounds); its time per round, times the rounds the whole block
 * takes, is the prediction.  When the best prediction is at most 500 ms, the
 * shapes predicted within 6 % of it (at most three) are then timed on the
 * whole block (the faster of two launches each), and the fastest is kept.
 * cache_path (when NULL, the environment variable
 * RAYSH_AUTOTUNE_CACHE; no cache if both are unset) names a text file of
 * earlier choices keyed by GPU architecture, CU count, HIP runtime version,
 * precision and log2(n_stars): a hit skips the timing, a miss appends a
 * line.  Synchronous.  Errors as raysh_map; ENOMEM if the scratch map cannot
 * be allocated.
 */
int raysh_autotune(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix, int precision,
                   const char *cache_path, int *cx, int *cy, int *share, int *star_tile);

/*
 * raysh_autotune_batch: the launch shape of raysh_map_batch for these sets
 * (arrays of length n_sets, as raysh_map_batch takes them): every shape
 * compiled for `precision` is timed with the persistent batch kernel on a
 * sample batch made of a central block of each set's rays (about an equal
 * share of 1e11 ray-star interactions per set, sides in whole multiples of
 * 128 rays so that no compiled tile is ragged in it, at most the block),
 * mapped into scratch maps; the fastest is set in every
 * context (raysh_map_batch uses the shape of sets[0]) and returned through
 * the optional out-pointers.  The cache is that of raysh_autotune, keyed
 * also by "batch" and by the mean star count of the sets.  Synchronous.
 * Errors as raysh_map_batch; ENOMEM if the scratch maps cannot be
 * allocated.  On error the contexts keep their shapes.
 */
int raysh_autotune_batch(raysh_ctx *const *sets, int n_sets, const raysh_rays *rays, const raysh_pixels *pix,
                         int precision, const char *cache_path, int *cx, int *cy, int *share, int *star_tile);

/*
 * raysh_shoot: per-ray results of Eq. (1) for one block of rays.
 *   beta_x, beta_y: device FP64 arrays of nx*ny, element j*nx + i
 *                   (may be NULL); written with beta of ray (i, j).
 *   bin:            device int32 array of nx*ny (may be NULL, then pix may
 *                   be NULL); written with the linear pixel index
 *                   js*pix->nx + is, or -1 when the ray is dropped or
 *                   outside the window.
 * EINVAL on bad rays/pixels/precision, on a NULL ctx, or when an output
 * pointer is not device memory large enough for nx*ny elements;
 * EOVERFLOW when nx*ny > 2^31 - 1 or i0 + nx, j0 + ny > 2^53.
 * An empty block (nx or ny == 0) is a no-op.
 */
int raysh_shoot(raysh_ctx *ctx, const raysh_rays *rays, int precision,
                double *beta_x, double *beta_y, const raysh_pixels *pix, int32_t *bin);

/*
 * raysh_map: Algorithm 1 for one block of rays: ADDS one to counts[js*nx + is]
 * for every ray that lands in the window (the map is accumulated, never
 * cleared, so maps of disjoint blocks of one lattice sum to the map of the
 * whole lattice).  counts: device int32 [pix->ny][pix->nx].
 * n_binned (optional, HOST pointer): if not NULL, the call waits for the
 * stream and stores the number of rays this call binned.
 * Errors as raysh_shoot; EINVAL also when counts is NULL or not device
 * memory of nx*ny int32.  Counts wrap silently only if one pixel receives
 * more than 2^31 - 1 rays over several calls (one call cannot: its ray count
 * is below 2^31).
 */
int raysh_map(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix,
              int precision, int32_t *counts, uint64_t *n_binned);

/*
 * raysh_map_split_noalloc: raysh_map in RAYSH_FP64 with each ray's star sum
 * split over `parts` contiguous star ranges (as raysh_set_star_split; 0 =
 * automatic, 1 = one pass), for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  It allocates nothing and never synchronizes: the partial
 * sums (parts * nx * ny * 16 bytes) go to a static device array of 64 MiB
 * that the library holds on each device it runs on until the process ends
 * (its address is resolved by raysh_init).  Every call on a device shares
 * that array, so calls that overlap on one device race; each call writes
 * every partial sum it reads.  The map is accumulated, as in raysh_map, and
 * equals raysh_map's for the same split, bit for bit.
 * Errors as raysh_map; EINVAL when parts is outside [0, 65536]; EOVERFLOW
 * when the partial sums exceed 64 MiB (nothing is enqueued).
 */
int raysh_map_split_noalloc(raysh_ctx *ctx, const raysh_rays *rays, const raysh_pixels *pix, int parts,
                            int32_t *counts);

/*
 * raysh_map_batch: raysh_map for n_sets independent lenses in one launch
 * (Sec. 2.2 mentions grids of independent simulations over lens parameters).
 * sets[s] is a context (all on one device; the stream of sets[0] is used),
 * rays[s], pix[s] its lattice block and window, counts[s] its device map.
 * Work items (set, ray tile) are ordered longest first and drained by a
 * persistent grid from a device work queue; the launch is captured once into
 * a HIP graph per (sets, shapes) and replayed when the same batch is run again.
 * Maps are accumulated, as in raysh_map.  Errors: as raysh_map for every set,
 * EINVAL if n_sets < 1 or the contexts are on different devices.
 */
int raysh_map_batch(raysh_ctx *const *sets, int n_sets, const raysh_rays *rays,
                    const raysh_pixels *pix, int precision, int32_t *const *counts);

/* ----------------------------------------------------------------------
 * Learned surrogate: magnification histograms and a small network that
 * predicts them from lens parameters.  Ray counts per pixel are
 * proportional to magnification, and a finite source sees the map
 * convolved with its profile (Sec. 1); many maps over a parameter grid
 * feed the Bayesian Monte Carlo analysis the paper's introduction
 * describes.
 * ---------------------------------------------------------------------- */

/* Device workspace, in bytes, that raysh_log_mag_histogram needs for an
 * nx x ny map (0 for a non-positive size). */
size_t raysh_histogram_workspace(int32_t nx, int32_t ny);

/*
 * raysh_log_mag_histogram: histogram of log10(mu_sigma / mu_ref) over a map.
 *   counts: device int32 map [ny][nx] (as written by raysh_map);
 *   norm:   (dx*dy)/(px*py) of the lattice and window, so that
 *           mu = counts * norm is the magnification;
 *   sigma:  width of the circular Gaussian source, in angle units; the
 *           profile is sampled at pixel offsets |k| <= ceil(3 sigma / p),
 *           normalised per axis and applied separably; only pixels at least
 *           that far from every edge are counted;
 *   bins:   nbins uniform bins on [lo, hi); values below lo (mu_sigma = 0
 *           too) go to the first bin, values at or above hi to the last.
 * Outputs (device): bin_counts uint32[nbins] (overwritten) and, if not NULL,
 * hist float[nbins] = bin_counts / their sum.  workspace: device memory of
 * raysh_histogram_workspace(nx, ny) bytes.  All arithmetic is FP64.
 * Asynchronous on hip_stream (NULL = null stream), on the counts' device.
 * EINVAL on a bad size, range or pointer, or when no pixel lies 3 sigma
 * inside the map; EOVERFLOW above 2^31-1 pixels.
 */
int raysh_log_mag_histogram(const int32_t *counts, int32_t nx, int32_t ny, double norm, double sigma,
                            double px, double py, double mu_ref, int32_t nbins, double lo, double hi,
                            void *workspace, size_t workspace_bytes, uint32_t *bin_counts, float *hist,
                            void *hip_stream);

/* ------------------------------------------------------------------------
 * Simulated light curves.  A magnification map and a model of the source's
 * size and brightness profile give simulated light curves, which the
 * Bayesian Monte Carlo analysis compares with observed ones (Sec. 1).  The
 * paper fixes neither the profile nor the tracks; the library offers the two
 * profiles below and straight tracks.
 * ---------------------------------------------------------------------- */
enum {
    RAYSH_SOURCE_GAUSSIAN = 0,  /* circular Gaussian of width `size`: taps at
                                   pixel offsets |k| <= r = ceil(3 size / p),
                                   normalised per axis, applied rows then
                                   columns (as raysh_log_mag_histogram) */
    RAYSH_SOURCE_DISK = 1       /* uniform disk of radius `size`: the pixels at
                                   offsets (k, l) with (k px)^2 + (l py)^2 <=
                                   size^2 in FP64; the value is (norm * S) / n,
                                   S the integer sum of their counts, n their
                                   number; rx, ry are the largest |k| on row 0
                                   and |l| on column 0 in the disk */
};

/* Half-widths (rx, ry) of a profile on a map of nx x ny pixels of size
 * px x py; the source map has (nx - 2 rx) x (ny - 2 ry) pixels.  rx, ry may
 * be NULL.  EINVAL on an unknown profile, a size, pixel or map size that is
 * not finite and > 0, a source whose reach (3 size for the Gaussian, size
 * for the disk) is not below nx px and ny py, or a source map smaller than
 * 2 x 2 pixels. */
int raysh_source_map_shape(int32_t nx, int32_t ny, int profile, double size, double px, double py,
                           int32_t *rx, int32_t *ry);

/* Device workspace, in bytes, that raysh_source_map needs (0 for a
 * non-positive size). */
size_t raysh_source_map_workspace(int32_t nx, int32_t ny);

/*
 * raysh_source_map: the magnification map seen by a source of the given
 * profile.  counts: device int32 map [ny][nx] (as written by raysh_map);
 * norm = (dx*dy)/(px*py), so that counts * norm is the magnification.
 * mu_s: device FP64 [ny - 2 ry][nx - 2 rx]; its pixel (i, j) is pixel
 * (i + rx, j + ry) of the map, so its own grid starts at
 * (x0 + rx px, y0 + ry py) of the map's window.  All arithmetic is FP64.
 * workspace: device memory of raysh_source_map_workspace(nx, ny) bytes.
 * Asynchronous on hip_stream (NULL = null stream), on the counts' device.
 * Errors as raysh_source_map_shape, plus EINVAL on NULL or non-device
 * buffers, a short workspace or a norm that is not finite and > 0, and
 * EOVERFLOW above 2^31-1 pixels.
 */
int raysh_source_map(const int32_t *counts, int32_t nx, int32_t ny, double norm, int profile, double size,
                     double px, double py, void *workspace, size_t workspace_bytes, double *mu_s,
                     void *hip_stream);

/*
 * raysh_light_curves: n_tracks straight tracks across a source map.
 *   mu_s:  device FP64 [grid->ny][grid->nx]; its values sit at the pixel
 *          centres (grid->x0 + (i + 0.5) grid->px, grid->y0 + (j + 0.5) grid->py);
 *          grid->nx, grid->ny >= 2;
 *   track t runs from (xa[t], ya[t]) to (xb[t], yb[t]) (device FP64 arrays
 *          of n_tracks, source-plane angles) and is sampled at n_samples
 *          evenly spaced points, in the map's centre-index space: with
 *          ipx = 1 / grid->px and inv = 1 / (n_samples - 1) (0 when
 *          n_samples == 1), each rounded once,
 *            u_k = ((xa - x0) ipx - 0.5) + (((xb - xa) ipx) inv) k,
 *          likewise v_k with y, y0 and py;
 *   curves: device FP64 [n_tracks][n_samples]: a sample with
 *          0 <= u <= nx - 1 and 0 <= v <= ny - 1 takes the bilinear
 *          interpolation of its four surrounding centres (i = min(floor(u),
 *          nx - 2), fx = u - i, r0 = m[j][i] + fx (m[j][i+1] - m[j][i]),
 *          r1 likewise on row j+1, value r0 + fy (r1 - r0)); any other
 *          sample is NaN.  Every product and sum is rounded on its own;
 *   order: NULL (tracks in the order given) or device int32[n_tracks], a
 *          permutation of the tracks in which to visit them (as written by
 *          raysh_track_order).  The curves are the same either way: row t
 *          of curves is track t.  Entries outside [0, n_tracks) are skipped;
 *   sorted: NULL, or (with order) device FP64[4][n_tracks]: the end points
 *          xa, ya, xb, yb in visiting order (as written by
 *          raysh_track_order), read in place of xa[order[i]] etc.; faster
 *          because they are read beside the order instead of after it.
 * Asynchronous on hip_stream, on mu_s's device.  n_tracks == 0 is a no-op.
 * EINVAL on a bad grid, n_tracks < 0, n_samples outside [1, 2^24], NULL or
 * non-device buffers, or sorted without order; EOVERFLOW above 2^31-1 map
 * pixels or (2^31-1) * 1024 samples.
 */
int raysh_light_curves(const double *mu_s, const raysh_pixels *grid, int64_t n_tracks, int32_t n_samples,
                       const double *xa, const double *ya, const double *xb, const double *yb,
                       const int32_t *order, const double *sorted, double *curves, void *hip_stream);

/* Device workspace, in bytes, that raysh_track_order needs for a source map
 * of pixel grid `grid` (0 for an invalid grid). */
size_t raysh_track_order_workspace(const raysh_pixels *grid);

/*
 * raysh_track_order: a visiting order for raysh_light_curves in which tracks
 * that run together read neighbouring parts of the source map: the tracks
 * sorted by the cell (16 x 16 pixels of grid, larger for maps of more than
 * 2048 cells a side) holding the midpoint of their end points, cells in Z
 * (Morton) order; midpoints outside the map go to the nearest edge cell.  The
 * order of tracks within a cell is unspecified.
 *   xa, ya, xb, yb: device FP64 arrays of n_tracks end points (as for
 *                   raysh_light_curves);
 *   order:          device int32[n_tracks], overwritten with a permutation
 *                   of 0 .. n_tracks - 1;
 *   sorted:         NULL, or device FP64[4][n_tracks], overwritten with the
 *                   end points in that order (xa[order[i]] at [0][i],
 *                   ya at [1][i], xb at [2][i], yb at [3][i]);
 *   workspace:      device memory of raysh_track_order_workspace(grid) bytes.
 * Asynchronous on hip_stream, on xa's device.  n_tracks == 0 is a no-op.
 * EINVAL on a bad grid, n_tracks < 0, NULL or non-device buffers or a short
 * workspace; EOVERFLOW above 2^31-1 tracks.
 */
int raysh_track_order(const raysh_pixels *grid, int64_t n_tracks, const double *xa, const double *ya,
                      const double *xb, const double *yb, void *workspace, size_t workspace_bytes, int32_t *order,
                      double *sorted, void *hip_stream);

/*
 * The network: layers n_in -> n_hidden -> n_hidden -> n_out, GELU (erf
 * form) after the first two, softmax output.  Weights are used in BF16,
 * rounded to nearest-even from FP32 master copies; activations and sums are
 * FP32.  Parameters are FP32, flat: W1[n_in][n_hidden], b1[n_hidden],
 * W2[n_hidden][n_hidden], b2[n_hidden], W3[n_hidden][n_out], b3[n_out].
 */
typedef struct raysh_mlp raysh_mlp;

/* Create the network on `device`, work on hip_stream, with host initial
 * parameters `params` (copied) and room for batches up to max_batch.
 * EINVAL on sizes < 1 or > 4096 (max_batch > 2^20), NULL or non-finite
 * params; ENOMEM; EDEVICE. */
int raysh_mlp_create(raysh_mlp **out, int device, void *hip_stream, int32_t n_in, int32_t n_hidden,
                     int32_t n_out, int32_t max_batch, const float *params);

/* Number of parameters (0 for NULL). */
int64_t raysh_mlp_n_params(const raysh_mlp *mlp);

/* Copy the FP32 master parameters to host memory (synchronous). */
int raysh_mlp_get_params(const raysh_mlp *mlp, float *params);

/* Softmax outputs for x (device float[batch][n_in]) into probs (device
 * float[batch][n_out]); 1 <= batch <= max_batch. */
int raysh_mlp_forward(raysh_mlp *mlp, const float *x, int32_t batch, float *probs);

/* Cross-entropy -mean_b sum_j target_bj log p_bj against target (device
 * float[batch][n_out]) and its gradient with respect to the parameters,
 * kept for raysh_mlp_adam_step and, if grads (device float[n_params]) is not
 * NULL, copied there; loss (device float, may be NULL) receives the loss.
 * The BF16 rounding of the weights is passed straight through. */
int raysh_mlp_gradient(raysh_mlp *mlp, const float *x, const float *target, int32_t batch, float *grads,
                       float *loss);

/* One bias-corrected Adam step with the last gradient. */
int raysh_mlp_adam_step(raysh_mlp *mlp, float lr, float beta1, float beta2, float eps);

/* raysh_mlp_gradient followed by raysh_mlp_adam_step. */
int raysh_mlp_train_step(raysh_mlp *mlp, const float *x, const float *target, int32_t batch, float lr,
                         float beta1, float beta2, float eps, float *loss);

/* Wait for the network's work; release it (NULL is a no-op). */
int raysh_mlp_sync(raysh_mlp *mlp);
int raysh_mlp_free(raysh_mlp *mlp);

/*
 * raysh_fma_probe: a measurement aid for profilers, not part of the method.
 * Runs n_blocks workgroups of 256 threads; each thread keeps 8 independent
 * chains a <- fma(a, 1, 1) for n_iter steps and stores the sum of its chains
 * in out[block * 256 + thread] (device memory: double for RAYSH_FP64, float
 * for RAYSH_FP32_BULK).  Each wave issues exactly 8 * n_iter FMA
 * instructions of that precision and 7 adds, so a counter of FMA
 * instructions and the achieved FMA rate can be checked against known
 * numbers.  Every step is exact: thread t stores
 * sum over i < 8 of ((t mod 64) + i + n_iter).  Asynchronous on hip_stream,
 * on out's device.  EINVAL on another precision, n_blocks outside
 * [1, 2^31-1], n_iter < 1, or a NULL, non-device or short buffer.
 */
int raysh_fma_probe(int precision, int64_t n_blocks, int32_t n_iter, void *out, void *hip_stream);

/* Wait for all work enqueued by the context. */
int raysh_sync(raysh_ctx *ctx);

/* Release a context (waits for its work first).  NULL is a no-op. */
int raysh_free(raysh_ctx *ctx);

/* Message for the calling thread's last error ("" if none). */
const char *raysh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RAYSH_H */
