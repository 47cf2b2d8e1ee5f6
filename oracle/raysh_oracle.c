/*
 * raysh oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of backward ray
 * shooting through a random star field, written from Chen, Kantowski, Dai,
 * Baron & Van der Mark (2017), "Accelerating gravitational microlensing
 * simulations using the Xeon Phi coprocessor" (arXiv:1703.09707).
 *
 * What is computed is a composition of two maps, applied to every ray of a
 * regular image-plane lattice:
 *   - the lens map theta -> beta of Sec. 1, Eq. (2)-(3):
 *       beta = theta - alpha(theta),
 *       alpha(theta) = K theta + sum_k m_k (theta - theta_k) / |theta - theta_k|^2,
 *       K = [[kappa_c + gamma_1, gamma_2], [gamma_2, kappa_c - gamma_1]];
 *   - the pixel function beta -> (i_s, j_s) of the source-plane window,
 *     undefined (the ray is not counted) outside the window.
 * The magnification map of Algorithm 1 (Sec. 2.2) is the histogram of the
 * pixel function over the lattice's rays: mag[j_s][i_s] is the number of
 * rays whose source position falls in pixel (i_s, j_s).  Within alpha the
 * smooth term comes first and the stars follow in index order, each
 * operation one IEEE-rounded step.
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
 *   - a ray whose beta is not finite (it hit a star exactly) is not counted.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* The lens of Eq. (1): smooth convergence, shear and the point masses. */
typedef struct {
    double kappa_c, gamma1, gamma2;
    int64_t n_stars;
    const double *xs, *ys, *ms;
} lens_t;

/* The source-plane window and its pixels. */
typedef struct {
    double X0, Y0, Px, Py;
    int64_t NX, NY;
} window_t;

/* Image angle of lattice index idx (cell-centred). */
static double image_angle(double origin, int64_t idx, double step)
{
    double t = (double)idx + 0.5;
    t = t * step;
    return origin + t;
}

/* The lens map, Eq. (2)-(3): beta = theta - alpha(theta). */
static void lens_map(const lens_t *L, double tx, double ty, double *bx, double *by)
{
    /* smooth matter and shear: K theta */
    double ax = (L->kappa_c + L->gamma1) * tx + L->gamma2 * ty;
    double ay = L->gamma2 * tx + (L->kappa_c - L->gamma1) * ty;
    /* the point masses, in index order */
    for (int64_t k = 0; k < L->n_stars; ++k) {
        double ex = tx - L->xs[k];
        double ey = ty - L->ys[k];
        double r2 = ex * ex + ey * ey;
        double w = L->ms[k] / r2;
        ax += w * ex;
        ay += w * ey;
    }
    *bx = tx - ax;
    *by = ty - ay;
}

/* The pixel function: linear index js*NX + is of the pixel holding beta, or
 * -1 when beta is not finite or lies outside the window. */
static int64_t pixel_of(const window_t *W, double bx, double by)
{
    if (!isfinite(bx) || !isfinite(by))
        return -1;
    double u = (bx - W->X0) / W->Px;
    double v = (by - W->Y0) / W->Py;
    if (!(u >= 0.0 && u < (double)W->NX && v >= 0.0 && v < (double)W->NY))
        return -1;
    int64_t is = (int64_t)floor(u);
    int64_t js = (int64_t)floor(v);
    return js * W->NX + is;
}

static lens_t make_lens(double kappa_c, double gamma1, double gamma2, int64_t n_stars,
                        const double *xs, const double *ys, const double *ms)
{
    lens_t L = {kappa_c, gamma1, gamma2, n_stars, xs, ys, ms};
    return L;
}

static window_t make_window(double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY)
{
    window_t W = {X0, Y0, Px, Py, NX, NY};
    return W;
}

/*
 * The lens map and the pixel function at every ray of the nx-by-ny block of
 * the lattice whose global indices start at (i0, j0).  Outputs are j-major
 * (index j*nx + i); any output pointer may be NULL.
 */
void ora_shoot(double kappa_c, double gamma1, double gamma2,
               int64_t n_stars, const double *xs, const double *ys, const double *ms,
               double x0, double y0, double dx, double dy,
               int64_t nx, int64_t ny, int64_t i0, int64_t j0,
               double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
               double *beta_x, double *beta_y, int64_t *bin)
{
    const lens_t L = make_lens(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms);
    const window_t W = make_window(X0, Y0, Px, Py, NX, NY);
    for (int64_t j = 0; j < ny; ++j) {
        for (int64_t i = 0; i < nx; ++i) {
            double bx, by;
            lens_map(&L, image_angle(x0, i0 + i, dx), image_angle(y0, j0 + j, dy), &bx, &by);
            int64_t o = j * nx + i;
            if (beta_x) beta_x[o] = bx;
            if (beta_y) beta_y[o] = by;
            if (bin) bin[o] = pixel_of(&W, bx, by);
        }
    }
}

/*
 * The magnification map of the block: adds to counts[p] the number of rays
 * whose pixel is p (the map is accumulated, not cleared).  Returns the
 * number of rays counted.
 */
int64_t ora_map(double kappa_c, double gamma1, double gamma2,
                int64_t n_stars, const double *xs, const double *ys, const double *ms,
                double x0, double y0, double dx, double dy,
                int64_t nx, int64_t ny, int64_t i0, int64_t j0,
                double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
                int32_t *counts)
{
    const lens_t L = make_lens(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms);
    const window_t W = make_window(X0, Y0, Px, Py, NX, NY);
    int64_t counted = 0;
    for (int64_t j = 0; j < ny; ++j) {
        for (int64_t i = 0; i < nx; ++i) {
            double bx, by;
            lens_map(&L, image_angle(x0, i0 + i, dx), image_angle(y0, j0 + j, dy), &bx, &by);
            int64_t p = pixel_of(&W, bx, by);
            if (p >= 0) {
                counts[p] += 1;
                ++counted;
            }
        }
    }
    return counted;
}

/*
 * The lens map and the pixel function at an arbitrary list of rays given by
 * global lattice indices (ii[r], jj[r]); used to check sampled rays of large
 * lattices one by one.
 */
void ora_shoot_list(double kappa_c, double gamma1, double gamma2,
                    int64_t n_stars, const double *xs, const double *ys, const double *ms,
                    double x0, double y0, double dx, double dy,
                    int64_t n, const int64_t *ii, const int64_t *jj,
                    double X0, double Y0, double Px, double Py, int64_t NX, int64_t NY,
                    double *beta_x, double *beta_y, int64_t *bin)
{
    const lens_t L = make_lens(kappa_c, gamma1, gamma2, n_stars, xs, ys, ms);
    const window_t W = make_window(X0, Y0, Px, Py, NX, NY);
    for (int64_t r = 0; r < n; ++r) {
        double bx, by;
        lens_map(&L, image_angle(x0, ii[r], dx), image_angle(y0, jj[r], dy), &bx, &by);
        if (beta_x) beta_x[r] = bx;
        if (beta_y) beta_y[r] = by;
        if (bin) bin[r] = pixel_of(&W, bx, by);
    }
}

/*
 * The scale of the rounding errors of beta at one ray:
 *   S = |theta|_inf + |K theta|_inf + sum_k m_k / r_k,
 * the largest magnitude any term of beta = theta - K theta - sum_k (...)
 * can take (each star term has length m_k / r_k).  Per-ray tolerances on
 * beta are stated relative to it; by the triangle inequality |beta|_inf <= S.
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
