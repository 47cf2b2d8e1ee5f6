/*
 * raysh oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of backward ray
 * shooting through a random star field, written from Chen, Kantowski, Dai,
 * Baron & Van der Mark (2017), "Accelerating gravitational microlensing
 * simulations using the Xeon Phi coprocessor" (arXiv:1703.09707):
 *   - the lens equation, Sec. 1, Eq. (1)-(3): beta = theta - alpha, with
 *     alpha = K theta + sum_k m_k (theta - theta_k) / |theta - theta_k|^2 and
 *     K = [[kappa_c + gamma_1, gamma_2], [gamma_2, kappa_c - gamma_1]];
 *   - the per-ray steps of Algorithm 1 (Sec. 2.2), in its order: image
 *     angle, macro term, star sum in index order, source angle, pixel, count.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header or constant
 * with the GPU library.  Build with -O2 -fno-fast-math -ffp-contract=off so
 * that every operation below is one correctly rounded IEEE operation.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - a ray sits at the centre of its lattice cell: theta = origin + (idx + 1/2) * step,
 *     computed as ((double)idx + 0.5), times step, plus origin;
 *   - pixel (is, js) covers [X0 + is*Px, X0 + (is+1)*Px) x [Y0 + js*Py, ...);
 *     the pixel coordinate is (beta - X0) / Px with IEEE division, the window
 *     test is done in FP64 before the integer conversion, and the map is
 *     row-major with row js (the paper's mag[j_s, i_s]);
 *   - a ray whose beta is not finite (it hit a star exactly) is dropped.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* Image angle of lattice index idx (cell-centred). */
static double image_angle(double origin, int64_t idx, double step)
{
    double t = (double)idx + 0.5;
    t = t * step;
    return origin + t;
}

/* Eq. (3) then Eq. (2) for one ray: returns beta = theta - alpha. */
static void lens_one_ray(double kappa_c, double gamma1, double gamma2,
                         int64_t n_stars, const double *xs, const double *ys,
                         const double *ms, double tx, double ty,
                         double *bx, double *by)
{
    /* first term of Eq. (3): the smooth matter and shear */
    double ax = (kappa_c + gamma1) * tx + gamma2 * ty;
    double ay = gamma2 * tx + (kappa_c - gamma1) * ty;
    /* second term of Eq. (3): the stars, in index order */
    for (int64_t k = 0; k < n_stars; ++k) {
        double ex = tx - xs[k];
        double ey = ty - ys[k];
        double r2 = ex * ex + ey * ey;
        double w = ms[k] / r2;
        ax += w * ex;
        ay += w * ey;
    }
    /* Eq. (2) */
    *bx = tx - ax;
    *by = ty - ay;
}

/* Linear pixel index js*NX + is of a source angle, or -1 when the ray is
 * dropped (non-finite) or lands outside the source window. */
static int64_t pixel_index(double bx, double by, double X0, double Y0,
                           double Px, double Py, int64_t NX, int64_t NY)
{
    if (!isfinite(bx) || !isfinite(by))
        return -1;
    double u = (bx - X0) / Px;
    double v = (by - Y0) / Py;
    if (!(u >= 0.0 && u < (double)NX && v >= 0.0 && v < (double)NY))
        return -1;
    int64_t is = (int64_t)floor(u);
    int64_t js = (int64_t)floor(v);
    return js * NX + is;
}

/*
 * Per-ray source angles and pixel indices for the nx-by-ny block of rays
 * whose global lattice indices start at (i0, j0).  Outputs are j-major
 * (index j*nx + i); any output pointer may be NULL.
 */
void ora_shoot(double kappa_c, double gamma1, double gamma2,
               int64_t n_stars, const double *xs, const double *ys, const double *ms,
               double x0, double y0, double dx, double dy,
               int64_t nx, int64_t ny, int64_t i0, int64_t j0,
               double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
               double *beta_x, double *beta_y, int64_t *bin)
{
    for (int64_t j = 0; j < ny; ++j) {
        double ty = image_angle(y0, j0 + j, dy);
        for (int64_t i = 0; i < nx; ++i) {
            double tx = image_angle(x0, i0 + i, dx);
            double bx, by;
            lens_one_ray(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms, tx, ty, &bx, &by);
            int64_t o = j * nx + i;
            if (beta_x) beta_x[o] = bx;
            if (beta_y) beta_y[o] = by;
            if (bin) bin[o] = pixel_index(bx, by, X0, Y0, Px, Py, NX, NY);
        }
    }
}

/*
 * Algorithm 1 proper: adds one count per ray to counts[js*NX + is] (the map
 * is accumulated, not cleared).  Returns the number of rays binned.
 */
int64_t ora_map(double kappa_c, double gamma1, double gamma2,
                int64_t n_stars, const double *xs, const double *ys, const double *ms,
                double x0, double y0, double dx, double dy,
                int64_t nx, int64_t ny, int64_t i0, int64_t j0,
                double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
                int32_t *counts)
{
    int64_t binned = 0;
    for (int64_t j = 0; j < ny; ++j) {
        double ty = image_angle(y0, j0 + j, dy);
        for (int64_t i = 0; i < nx; ++i) {
            double tx = image_angle(x0, i0 + i, dx);
            double bx, by;
            lens_one_ray(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms, tx, ty, &bx, &by);
            int64_t p = pixel_index(bx, by, X0, Y0, Px, Py, NX, NY);
            if (p >= 0) {
                counts[p] += 1;
                ++binned;
            }
        }
    }
    return binned;
}

/*
 * Source angles of an arbitrary list of rays given by global lattice
 * indices (ii[r], jj[r]); used to check sampled rays of large grids one
 * by one.
 */
void ora_shoot_list(double kappa_c, double gamma1, double gamma2,
                    int64_t n_stars, const double *xs, const double *ys, const double *ms,
                    double x0, double y0, double dx, double dy,
                    int64_t n, const int64_t *ii, const int64_t *jj,
                    double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
                    double *beta_x, double *beta_y, int64_t *bin)
{
    for (int64_t r = 0; r < n; ++r) {
        double tx = image_angle(x0, ii[r], dx);
        double ty = image_angle(y0, jj[r], dy);
        double bx, by;
        lens_one_ray(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms, tx, ty, &bx, &by);
        if (beta_x) beta_x[r] = bx;
        if (beta_y) beta_y[r] = by;
        if (bin) bin[r] = pixel_index(bx, by, X0, Y0, Px, Py, NX, NY);
    }
}

/*
 * The rounding-error scale S = |theta|_inf + |K theta|_inf + sum_k m_k / r_k
 * of one ray; per-ray tolerances on beta are stated relative to it.
 */
double ora_error_scale(double kappa_c, double gamma1, double gamma2,
                       int64_t n_stars, const double *xs, const double *ys, const double *ms,
                       double tx, double ty)
{
    double ax = fabs((kappa_c + gamma1) * tx + gamma2 * ty);
    double ay = fabs(gamma2 * tx + (kappa_c - gamma1) * ty);
    double s = fmax(fabs(tx), fabs(ty)) + fmax(ax, ay);
    for (int64_t k = 0; k < n_stars; ++k) {
        double ex = tx - xs[k];
        double ey = ty - ys[k];
        s += ms[k] / sqrt(ex * ex + ey * ey);
    }
    return s;
}

/* error scale of every ray of a lattice block, j-major */
void ora_error_scale_block(double kappa_c, double gamma1, double gamma2,
                           int64_t n_stars, const double *xs, const double *ys, const double *ms,
                           double x0, double y0, double dx, double dy,
                           int64_t nx, int64_t ny, int64_t i0, int64_t j0, double *scale)
{
    for (int64_t j = 0; j < ny; ++j) {
        double ty = image_angle(y0, j0 + j, dy);
        for (int64_t i = 0; i < nx; ++i) {
            double tx = image_angle(x0, i0 + i, dx);
            scale[j * nx + i] = ora_error_scale(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms, tx, ty);
        }
    }
}
