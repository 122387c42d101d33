/*
 * FP64 direct evaluation of the discrete photoionization sum (oracle; test
 * infrastructure only -- the GPU library never links or calls this file).
 *
 * Computes, for each requested target cell t of a uniform nx*ny*nz grid,
 *     S_t = sum_j G(x_t, y_j) q_j
 * with G the discrete kernel of Section 3 (after eq. (summation)): the midpoint
 * value g(R)/(4 pi R^2) for j != t and the 2x2x2 Gauss-Legendre self value for
 * j == t, g from eq. (gfun).  q_j already carries the cell volume.
 *
 * Cell offsets are integers, so R = sqrt((di hx)^2 + (dj hy)^2 + (dk hz)^2) is
 * formed from exact integer differences.  The exponential difference is
 * evaluated as -exp(-aR)*expm1(-(b-a)R).  Each target's sum runs over the
 * sources in grid order (x slowest, z fastest), accumulating one z-row at a time
 * and then adding the row to the total, so the result does not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static double kernel_k(double R, double a, double b, double inv4piln)
{
    return -exp(-a * R) * expm1(-(b - a) * R) * inv4piln / (R * R * R);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_direct_targets(int32_t nx, int32_t ny, int32_t nz,
                           double hx, double hy, double hz,
                           const double *q, double a, double b, double ln_ratio,
                           const int64_t *tgt, int64_t nt, double *out)
{
    const double inv4piln = 1.0 / (4.0 * M_PI * ln_ratio);
    const double s2 = hx * hx + hy * hy + hz * hz;
    const double rho = sqrt(s2 / 12.0);
    /* 3 g(rho) / (pi s2), g(r) = (e^{-ar} - e^{-br}) / (r ln) */
    const double gself = -exp(-a * rho) * expm1(-(b - a) * rho) / (rho * ln_ratio);
    const double self = 3.0 * gself / (M_PI * s2);
    const int64_t nyz = (int64_t)ny * nz;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t it = tgt[t] / nyz;
        const int64_t jt = (tgt[t] / nz) % ny;
        const int64_t kt = tgt[t] % nz;
        double total = 0.0;
        for (int64_t i = 0; i < nx; ++i) {
            const double dx = (double)(i - it) * hx;
            for (int64_t j = 0; j < ny; ++j) {
                const double dy = (double)(j - jt) * hy;
                const double *qr = q + (i * ny + j) * nz;
                double row = 0.0;
                for (int64_t k = 0; k < nz; ++k) {
                    const double dz = (double)(k - kt) * hz;
                    const double R2 = dx * dx + dy * dy + dz * dz;
                    if (R2 == 0.0)
                        row += self * qr[k];
                    else
                        row += kernel_k(sqrt(R2), a, b, inv4piln) * qr[k];
                }
                total += row;
            }
        }
        out[t] = total;
    }
}
