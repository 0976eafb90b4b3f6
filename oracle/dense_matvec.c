/*
 * Dense direct DDA matrix-vector product, FP64, plain C + OpenMP.
 *
 * TEST INFRASTRUCTURE (oracle): used only by the tests, the smoke check and
 * the benchmark's CPU-baseline leg.  It shares nothing with the HIP library.
 *
 * For occupied dipoles i = 0..n-1 at centres r_i (nm):
 *
 *   mode 0:  y_i = x_i / alpha_i - sum_{j != i} G(r_i - r_j) x_j
 *   mode 1:  y_i =                 sum_{j != i} G(r_i - r_j) x_j
 *
 * with the point-dipole interaction obtained from the Green's tensor of
 * eq. (5) (times 4 pi k^2, see oracle/interaction.py):
 *
 *   G(R) x = e^{ikR}/R^3 [ (k^2R^2 + ikR - 1) x + (3 - 3ikR - k^2R^2) Rh (Rh . x) ]
 *
 * Every pair is evaluated on the fly: O(n^2) work, no FFT, no blocking.
 * Layouts: centres [n][3] (x,y,z); alpha_inv [n] complex; x, y [n][3]
 * complex (component fastest), complex = two doubles (re, im).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void oracle_dense_matvec(int64_t n, const double *centres, const double *alpha_inv,
                         double k_re, double k_im, const double *x, double *y, int mode)
{
    const double complex k = k_re + I * k_im;
    const double complex *xc = (const double complex *)x;
    const double complex *ai = (const double complex *)alpha_inv;
    double complex *yc = (double complex *)y;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        const double xi = centres[3 * i], yi = centres[3 * i + 1], zi = centres[3 * i + 2];
        double complex s0 = 0, s1 = 0, s2 = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double Rx = xi - centres[3 * j];
            const double Ry = yi - centres[3 * j + 1];
            const double Rz = zi - centres[3 * j + 2];
            const double r = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
            const double complex kr = k * r;
            const double complex e = cexp(I * kr) / (r * r * r);
            const double complex a = e * (kr * kr + I * kr - 1.0);
            const double complex b = e * (3.0 - 3.0 * I * kr - kr * kr);
            const double hx = Rx / r, hy = Ry / r, hz = Rz / r;
            const double complex x0 = xc[3 * j], x1 = xc[3 * j + 1], x2 = xc[3 * j + 2];
            const double complex proj = b * (hx * x0 + hy * x1 + hz * x2);
            s0 += a * x0 + proj * hx;
            s1 += a * x1 + proj * hy;
            s2 += a * x2 + proj * hz;
        }
        if (mode == 0) {
            yc[3 * i] = xc[3 * i] * ai[i] - s0;
            yc[3 * i + 1] = xc[3 * i + 1] * ai[i] - s1;
            yc[3 * i + 2] = xc[3 * i + 2] * ai[i] - s2;
        } else {
            yc[3 * i] = s0;
            yc[3 * i + 1] = s1;
            yc[3 * i + 2] = s2;
        }
    }
}

int oracle_num_threads(void)
{
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}

/*
 * Selected rows of the same product: y[r] = (A x)_{rows[r]} (mode 0) or the
 * interaction part only (mode 1), for r < nrows.  y is [nrows][3] complex.
 * Lets large lattices be checked on sampled outputs in O(nrows * n) work.
 */
void oracle_dense_matvec_rows(int64_t n, const double *centres, const double *alpha_inv,
                              double k_re, double k_im, const double *x, const int64_t *rows,
                              int64_t nrows, double *y, int mode)
{
    const double complex k = k_re + I * k_im;
    const double complex *xc = (const double complex *)x;
    const double complex *ai = (const double complex *)alpha_inv;
    double complex *yc = (double complex *)y;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrows; ++q) {
        const int64_t i = rows[q];
        const double xi = centres[3 * i], yi = centres[3 * i + 1], zi = centres[3 * i + 2];
        double complex s0 = 0, s1 = 0, s2 = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double Rx = xi - centres[3 * j];
            const double Ry = yi - centres[3 * j + 1];
            const double Rz = zi - centres[3 * j + 2];
            const double r = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
            const double complex kr = k * r;
            const double complex e = cexp(I * kr) / (r * r * r);
            const double complex a = e * (kr * kr + I * kr - 1.0);
            const double complex b = e * (3.0 - 3.0 * I * kr - kr * kr);
            const double hx = Rx / r, hy = Ry / r, hz = Rz / r;
            const double complex x0 = xc[3 * j], x1 = xc[3 * j + 1], x2 = xc[3 * j + 2];
            const double complex proj = b * (hx * x0 + hy * x1 + hz * x2);
            s0 += a * x0 + proj * hx;
            s1 += a * x1 + proj * hy;
            s2 += a * x2 + proj * hz;
        }
        if (mode == 0) {
            yc[3 * q] = xc[3 * i] * ai[i] - s0;
            yc[3 * q + 1] = xc[3 * i + 1] * ai[i] - s1;
            yc[3 * q + 2] = xc[3 * i + 2] * ai[i] - s2;
        } else {
            yc[3 * q] = s0;
            yc[3 * q + 1] = s1;
            yc[3 * q + 2] = s2;
        }
    }
}
