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
//
// FP32 kernel values (direct_kernel_f32) are written for throughput on the VALU:
// 1/R from the hardware reciprocal square root (1/R^3 = rsq^3, no division),
// exponentials from the hardware base-2 exponential, and 1 - e^{-x}, x = (b-a)R,
// as 1 - exp2(-x log2 e) for x >= 1/2 and as its Taylor polynomial (degree 9,
// truncation below 1e-8 relative) for x < 1/2, where the difference would cancel.
// The self cell is a select, not a branch.
#include "common.h"

namespace kifmm {

namespace {

constexpr int kThreads = 256;

__device__ inline double pair_value(int di, int dj, int dk, double hx, double hy, double hz, double a, double bma,
                                    double c, double self) {
    const double dx = di * hx, dy = dj * hy, dz = dk * hz;
    const double R2 = dx * dx + dy * dy + dz * dz;
    if (R2 == 0.0) return self;
    const double R = sqrt(R2);
    return -exp(-a * R) * expm1(-bma * R) * c / (R2 * R);
}

// FP64 kernel values and sums
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
                    acc += pair_value(i - it, j - jt, k - kt, hx, hy, hz, a, bma, c, self) *
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

// FP32 kernel values, FP64 sums; rows of the source grid are split over the NT threads as
// in direct_kernel, with the row index kept as (i, j) to avoid 64-bit divisions.  Few
// targets get 1024-thread workgroups so that the 256 CUs still hold several waves each.
template <int NT>
__global__ __launch_bounds__(NT) void direct_kernel_f32(
    int nx, int ny, int nz, float hx, float hy, float hz, const float *__restrict__ I,
    const int64_t *__restrict__ tgt, int64_t ntgt, double scale, float aL2, float x_per_R, float xL2_per_R,
    float c, float self, double *__restrict__ out) {
    __shared__ double red[NT / 64];
    const int kper = nz < NT ? nz : NT;
    const int rows_per_iter = NT / kper;
    const int dr = threadIdx.x / kper;
    const int kk = threadIdx.x % kper;
    const int64_t nyz = (int64_t)ny * nz;
    // -expm1(-x) = x (1 - x/2 + x^2/6 - ...): coefficients of x^0 .. x^8 of the bracket
    const float q1 = -1.f / 2, q2 = 1.f / 6, q3 = -1.f / 24, q4 = 1.f / 120, q5 = -1.f / 720, q6 = 1.f / 5040,
                q7 = -1.f / 40320, q8 = 1.f / 362880;
    for (int64_t t = blockIdx.x; t < ntgt; t += gridDim.x) {
        const int64_t g = tgt ? tgt[t] : t;
        const int it = (int)(g / nyz), jt = (int)((g / nz) % ny), kt = (int)(g % nz);
        double acc = 0.0;
        if (dr < rows_per_iter) {
            int i = 0, j = dr;
            while (j >= ny) { j -= ny; ++i; }
            const float *Ir = I + ((int64_t)i * ny + j) * nz;
            while (i < nx) {
                const float dx = (float)(i - it) * hx, dy = (float)(j - jt) * hy;
                const float dxy2 = dx * dx + dy * dy;
                for (int k = kk; k < nz; k += kper) {
                    const float dz = (float)(k - kt) * hz;
                    const float R2 = fmaf(dz, dz, dxy2);
                    const bool diag = R2 == 0.f;
                    const float R2s = diag ? 1.f : R2;
                    const float rs = __builtin_amdgcn_rsqf(R2s);
                    const float R = R2s * rs;
                    const float ea = __builtin_amdgcn_exp2f(-aL2 * R);
                    const float x = x_per_R * R;
                    const float one_minus = 1.f - __builtin_amdgcn_exp2f(-xL2_per_R * R);
                    float poly = fmaf(q8, x, q7);
                    poly = fmaf(poly, x, q6);
                    poly = fmaf(poly, x, q5);
                    poly = fmaf(poly, x, q4);
                    poly = fmaf(poly, x, q3);
                    poly = fmaf(poly, x, q2);
                    poly = fmaf(poly, x, q1);
                    poly = fmaf(poly, x, 1.f);
                    const float d = x < 0.5f ? x * poly : one_minus;
                    const float v = diag ? self : ea * d * c * (rs * rs * rs);
                    acc += (double)(v * Ir[k]);
                }
                j += rows_per_iter;
                Ir += (int64_t)rows_per_iter * nz;
                while (j >= ny) { j -= ny; ++i; }
            }
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w];
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
        hipLaunchKernelGGL(direct_kernel, dim3(grid), dim3(kThreads), 0, st, g->nx, g->ny,
                           g->nz, g->hx, g->hy, g->hz, I, tgt, ntgt, scale, a, b - a, c, self, out);
    else if (ntgt < 2048)
        hipLaunchKernelGGL(direct_kernel_f32<1024>, dim3(grid), dim3(1024), 0, st, g->nx, g->ny, g->nz,
                           (float)g->hx, (float)g->hy, (float)g->hz, I, tgt, ntgt, scale,
                           (float)(a * M_LOG2E), (float)(b - a), (float)((b - a) * M_LOG2E), (float)c,
                           (float)self, out);
    else
        hipLaunchKernelGGL(direct_kernel_f32<kThreads>, dim3(grid), dim3(kThreads), 0, st, g->nx, g->ny,
                           g->nz, (float)g->hx, (float)g->hy, (float)g->hz, I, tgt, ntgt, scale,
                           (float)(a * M_LOG2E), (float)(b - a), (float)((b - a) * M_LOG2E), (float)c,
                           (float)self, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
