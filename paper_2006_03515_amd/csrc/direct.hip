// Direct evaluation of the discrete photoionization sum at chosen targets
// (Section 3, eq. (summation) with the discrete kernel G defined after it).
//
// One workgroup per target (grid-stride over targets).  The 256 threads sweep the
// sources in grid order: each thread owns a fixed z position inside a row and
// walks the (i, j) rows, so consecutive lanes read consecutive floats of I.
// Distances come from integer cell offsets times h, never from differences of
// absolute coordinates, and the exponential difference is evaluated as
// -exp(-aR) * expm1(-(b-a)R).  Per-thread sums are FP64; the block reduction
// is a fixed tree, so results are bitwise repeatable.
#include "common.h"

namespace kifmm {

namespace {

constexpr int kThreads = 256;

template <bool F64>
__device__ inline double pair_value(int di, int dj, int dk, double hx, double hy, double hz,
                                    double a, double bma, double c, double self) {
    if (F64) {
        const double dx = di * hx, dy = dj * hy, dz = dk * hz;
        const double R2 = dx * dx + dy * dy + dz * dz;
        if (R2 == 0.0) return self;
        const double R = sqrt(R2);
        return -exp(-a * R) * expm1(-bma * R) * c / (R2 * R);
    } else {
        const float dx = (float)di * (float)hx, dy = (float)dj * (float)hy, dz = (float)dk * (float)hz;
        const float R2 = dx * dx + dy * dy + dz * dz;
        if (R2 == 0.0f) return self;
        const float R = sqrtf(R2);
        return (double)(-expf(-(float)a * R) * expm1f(-(float)bma * R) * (float)c / (R2 * R));
    }
}

template <bool F64>
__global__ __launch_bounds__(kThreads) void direct_kernel(
    int nx, int ny, int nz, double hx, double hy, double hz, const float *__restrict__ I,
    const int64_t *__restrict__ tgt, int64_t ntgt, double scale, double a, double bma,
    double c, double self, double *__restrict__ out) {
    __shared__ double red[kThreads / 64];
    const int kper = nz < kThreads ? nz : kThreads;        // threads per row
    const int rows_per_iter = kThreads / kper;             // rows handled at once
    const int dr = threadIdx.x / kper;
    const int kk = threadIdx.x % kper;
    const int64_t nrows = (int64_t)nx * ny;
    const int64_t nyz = (int64_t)ny * nz;
    for (int64_t t = blockIdx.x; t < ntgt; t += gridDim.x) {
        const int64_t g = tgt ? tgt[t] : t;
        const int it = (int)(g / nyz), jt = (int)((g / nz) % ny), kt = (int)(g % nz);
        double acc = 0.0;
        if (dr < rows_per_iter) {
            for (int64_t row = dr; row < nrows; row += rows_per_iter) {
                const int i = (int)(row / ny), j = (int)(row % ny);
                const float *Ir = I + row * nz;
                for (int k = kk; k < nz; k += kper)
                    acc += pair_value<F64>(i - it, j - jt, k - kt, hx, hy, hz, a, bma, c, self) *
                           (double)Ir[k];
            }
        }
        // fixed-order reduction: wave shuffle then across waves
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) s += red[w];
            out[t] = s * scale;
        }
        __syncthreads();
    }
}

}  // namespace

int launch_direct(const kifmm_grid *g, const kifmm_kernel *k, const float *I, double prefactor,
                  const int64_t *tgt, int64_t ntgt, double *out, int fp64, hipStream_t st) {
    const double ln = std::log(k->chi_max / k->chi_min);
    const double a = k->chi_min * k->p_o2, b = k->chi_max * k->p_o2;
    const double c = 1.0 / (4.0 * M_PI * ln);
    const double s2 = g->hx * g->hx + g->hy * g->hy + g->hz * g->hz;
    const double rho = std::sqrt(s2 / 12.0);
    const double grho = -std::exp(-a * rho) * std::expm1(-(b - a) * rho) / (rho * ln);
    const double self = 3.0 * grho / (M_PI * s2);
    const double scale = prefactor * g->hx * g->hy * g->hz;
    if (ntgt == 0) return KIFMM_OK;
    const int64_t maxg = 1 << 20;
    const unsigned grid = (unsigned)(ntgt < maxg ? ntgt : maxg);
    if (fp64)
        hipLaunchKernelGGL(direct_kernel<true>, dim3(grid), dim3(kThreads), 0, st, g->nx, g->ny,
                           g->nz, g->hx, g->hy, g->hz, I, tgt, ntgt, scale, a, b - a, c, self, out);
    else
        hipLaunchKernelGGL(direct_kernel<false>, dim3(grid), dim3(kThreads), 0, st, g->nx, g->ny,
                           g->nz, g->hx, g->hy, g->hz, I, tgt, ntgt, scale, a, b - a, c, self, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
