// FP64 device kernels of the operator precompute (Section 3: eq. (s2m), (s2l),
// (m2m), (m2l), (l2l) and the pseudo-inverse remark).
//
//   kmat_kernel       G between two point sets (batched over rigid shifts)
//   near_kernel       near-range matrices of a leaf against its 27 neighbours,
//                     from integer cell offsets, with the self-cell value
//   jacobi_round      one round of a one-sided (Hestenes) Jacobi SVD sweep,
//                     round-robin pairing, one workgroup per column pair
//   colnorm_kernel    singular values as the column norms after convergence
//   svd_gather        U^T (k x m) and W = V Sigma^-1 (n x k) of the kept columns
//   gemm_f64          batched row-major FP64 GEMM (LDS tiled)
//   cast_pad          FP64 -> FP32 / FP64 / BF16 / FP16 copies into padded layouts
#include "common.h"

namespace kifmm {

namespace {

struct KParams {
    double a, bma, c, self;  // a, b - a, 1/(4 pi ln(chi_max/chi_min)), self-cell value
};

__device__ inline double kval(double R2, const KParams &p) {
    if (R2 == 0.0) return p.self;
    const double R = sqrt(R2);
    return -exp(-p.a * R) * expm1(-p.bma * R) * p.c / (R2 * R);
}

// out[b][i][j] = G(X_i + sx_b, Y_j + sy_b); transposed: out[b][j][i]
__global__ void kmat_kernel(const double *__restrict__ X, int nX, const double *__restrict__ Y,
                            int nY, const double *__restrict__ sx, const double *__restrict__ sy,
                            int transpose, KParams p, double *__restrict__ out) {
    const int b = blockIdx.y;
    const int64_t total = (int64_t)nX * nY;
    const double ox = sx ? sx[3 * b] : 0.0, oy = sx ? sx[3 * b + 1] : 0.0, oz = sx ? sx[3 * b + 2] : 0.0;
    const double px = sy ? sy[3 * b] : 0.0, py = sy ? sy[3 * b + 1] : 0.0, pz = sy ? sy[3 * b + 2] : 0.0;
    double *o = out + (int64_t)b * total;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        if (transpose) { j = (int)(e / nX); i = (int)(e % nX); }
        else { i = (int)(e / nY); j = (int)(e % nY); }
        const double dx = (X[3 * i] + ox) - (Y[3 * j] + px);
        const double dy = (X[3 * i + 1] + oy) - (Y[3 * j + 1] + py);
        const double dz = (X[3 * i + 2] + oz) - (Y[3 * j + 2] + pz);
        o[e] = kval(dx * dx + dy * dy + dz * dz, p);
    }
}

// Near-range matrix of tap t (neighbour offset o_t in leaves): row = target cell
// li (C order in the leaf of ell x ell x ellz cells), column = source cell lj of the
// neighbour leaf.  Cell offset d = li - lj - (ell, ell, ellz) * o_t (integers),
// R = |(h dx, h dy, hz dz)|.
__global__ void near_kernel(int ell, int ellz, double h, double hz, const int *__restrict__ offs, KParams p,
                            double *__restrict__ out) {
    const int t = blockIdx.y;
    const int s = ell * ell * ellz;
    const int64_t total = (int64_t)s * s;
    const int ox = offs[3 * t], oy = offs[3 * t + 1], oz = offs[3 * t + 2];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int li = (int)(e / s), lj = (int)(e % s);
        const int ix = li / (ell * ellz), iy = (li / ellz) % ell, iz = li % ellz;
        const int jx = lj / (ell * ellz), jy = (lj / ellz) % ell, jz = lj % ellz;
        const double dx = (double)(ix - jx - ell * ox) * h;
        const double dy = (double)(iy - jy - ell * oy) * h;
        const double dz = (double)(iz - jz - ellz * oz) * hz;
        out[(int64_t)t * total + e] = kval(dx * dx + dy * dy + dz * dz, p);
    }
}

__device__ inline double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

// One round of the round-robin pairing of npad columns (npad even): slot 0 is
// fixed, slots 1..npad-1 rotate by `round`; pair k joins slots k and npad-1-k.
// A: column j of batch b at A + b*sA + j*ldA (length m[b]); V likewise (n[b]).
__global__ __launch_bounds__(256) void jacobi_round(double *__restrict__ A, double *__restrict__ V,
                                                    const int *__restrict__ mdim,
                                                    const int *__restrict__ ndim, int npad,
                                                    int ldA, int ldV, int64_t sA, int64_t sV,
                                                    int round, double tol,
                                                    unsigned long long *__restrict__ offmax) {
    __shared__ double sh[3][4];
    const int b = blockIdx.y;
    const int m = mdim[b], n = ndim[b];
    const int k = blockIdx.x;
    auto slot = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (npad - 1)) + 1; };
    int p = slot(k), q = slot(npad - 1 - k);
    if (p > q) { int t = p; p = q; q = t; }
    if (q >= n) return;
    double *ap = A + b * sA + (int64_t)p * ldA;
    double *aq = A + b * sA + (int64_t)q * ldA;
    double al = 0, be = 0, ga = 0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = ap[i], y = aq[i];
        al += x * x; be += y * y; ga += x * y;
    }
    al = block_sum(al, sh[0]);
    be = block_sum(be, sh[1]);
    ga = block_sum(ga, sh[2]);
    if (ga == 0.0 || al == 0.0 || be == 0.0) return;
    const double off = fabs(ga) / sqrt(al * be);
    if (threadIdx.x == 0) atomicMax(offmax + b, (unsigned long long)__double_as_longlong(off));
    if (off <= tol) return;
    const double zeta = (be - al) / (2.0 * ga);
    const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = ap[i], y = aq[i];
        ap[i] = c * x - s * y;
        aq[i] = s * x + c * y;
    }
    double *vp = V + b * sV + (int64_t)p * ldV;
    double *vq = V + b * sV + (int64_t)q * ldV;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = vp[i], y = vq[i];
        vp[i] = c * x - s * y;
        vq[i] = s * x + c * y;
    }
}

__global__ void colnorm_kernel(const double *__restrict__ A, const int *__restrict__ mdim,
                               const int *__restrict__ ndim, int ldA, int64_t sA, int npad,
                               double *__restrict__ sigma) {
    __shared__ double sh[4];
    const int b = blockIdx.y, j = blockIdx.x;
    const int m = mdim[b], n = ndim[b];
    if (j >= n) {
        if (threadIdx.x == 0) sigma[(int64_t)b * npad + j] = 0.0;
        return;
    }
    const double *a = A + b * sA + (int64_t)j * ldA;
    double v = 0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) v += a[i] * a[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) sigma[(int64_t)b * npad + j] = sqrt(v);
}

// UT[r][i] = A[:, order[r]][i] / sigma (r < k, i < m); W[i][r] = V[:, order[r]][i] / sigma
__global__ void svd_gather(const double *__restrict__ A, const double *__restrict__ V, int ldA,
                           int ldV, int m, int n, int k, const int *__restrict__ order,
                           const double *__restrict__ sig, double *__restrict__ UT,
                           double *__restrict__ W) {
    const int r = blockIdx.x;
    const int j = order[r];
    const double inv = 1.0 / sig[r];
    for (int i = threadIdx.x; i < m; i += blockDim.x) UT[(int64_t)r * m + i] = A[(int64_t)j * ldA + i] * inv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) W[(int64_t)i * k + r] = V[(int64_t)j * ldV + i] * inv;
}

// C[b] (M x N) = A[b] (M x K) * B[b] (K x N), row-major with leading dims; batch
// strides may be 0 (shared operand).
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void gemm_f64(int M, int N, int K, const double *__restrict__ A,
                                                int lda, int64_t sA, const double *__restrict__ B,
                                                int ldb, int64_t sB, double *__restrict__ C,
                                                int ldc, int64_t sC) {
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int b = blockIdx.z;
    A += b * sA; B += b * sB; C += b * sC;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int e = threadIdx.x; e < GT * GK; e += 256) {
            const int r = e / GK, kk = e % GK;
            const int gm = m0 + r, gk = k0 + kk;
            As[kk][r] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : 0.0;
            const int kk2 = e / GT, c = e % GT;
            const int gn = n0 + c, gk2 = k0 + kk2;
            Bs[kk2][c] = (gn < N && gk2 < K) ? B[(int64_t)gk2 * ldb + gn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double a[4], bb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
            if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = acc[i][j];
        }
}

template <typename T>
__device__ inline T from_double(double v);
template <> __device__ inline float from_double<float>(double v) { return (float)v; }
template <> __device__ inline double from_double<double>(double v) { return v; }
template <> __device__ inline __bf16 from_double<__bf16>(double v) { return (__bf16)(float)v; }
template <> __device__ inline _Float16 from_double<_Float16>(double v) { return (_Float16)(float)v; }

// dst[b][i][j] (Mp x Kp) = scale * src[b][i][j] (M x K), zero in the padding
template <typename T>
__global__ void cast_pad(const double *__restrict__ src, int M, int K, int64_t sS,
                         T *__restrict__ dst, int Mp, int Kp, int64_t sD, double scale) {
    const int b = blockIdx.y;
    const int64_t total = (int64_t)Mp * Kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / Kp), j = (int)(e % Kp);
        const double v = (i < M && j < K) ? src[b * sS + (int64_t)i * K + j] * scale : 0.0;
        dst[b * sD + e] = from_double<T>(v);
    }
}

// low part of a split-BF16 operand: dst = bf16(v - float(bf16(v))), v = scale * src
__global__ void cast_pad_lo(const double *__restrict__ src, int M, int K, int64_t sS,
                            __bf16 *__restrict__ dst, int Mp, int Kp, int64_t sD, double scale) {
    const int b = blockIdx.y;
    const int64_t total = (int64_t)Mp * Kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / Kp), j = (int)(e % Kp);
        const double v = (i < M && j < K) ? src[b * sS + (int64_t)i * K + j] * scale : 0.0;
        const float hi = (float)(__bf16)(float)v;
        dst[b * sD + e] = (__bf16)(float)(v - (double)hi);
    }
}

unsigned blocks_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

// ------------------------------------------------------------ launchers ----
// kernel parameters; the self-cell value of the discrete kernel (after eq. (summation)) for
// cells of h x h x hz
KParams make_params(const kifmm_kernel &k, double h, double hz) {
    const double ln = std::log(k.chi_max / k.chi_min);
    const double a = k.chi_min * k.p_o2, b = k.chi_max * k.p_o2;
    KParams p;
    p.a = a;
    p.bma = b - a;
    p.c = 1.0 / (4.0 * M_PI * ln);
    const double s2 = 2.0 * h * h + hz * hz;
    const double rho = std::sqrt(s2 / 12.0);
    const double grho = -std::exp(-a * rho) * std::expm1(-(b - a) * rho) / (rho * ln);
    p.self = 3.0 * grho / (M_PI * s2);
    return p;
}

int launch_kmat(const double *X, int nX, const double *Y, int nY, const double *sx,
                const double *sy, int batch, int transpose, const kifmm_kernel &k, double h,
                double *out, hipStream_t st) {
    KParams p = make_params(k, h, h);
    hipLaunchKernelGGL(kmat_kernel, dim3(blocks_for((int64_t)nX * nY), batch), dim3(256), 0, st,
                       X, nX, Y, nY, sx, sy, transpose, p, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_near(int ell, int ellz, double h, double hz, const int *offs_dev, int ntaps, const kifmm_kernel &k,
                double *out, hipStream_t st) {
    KParams p = make_params(k, h, hz);
    const int64_t s = (int64_t)ell * ell * ellz;
    hipLaunchKernelGGL(near_kernel, dim3(blocks_for(s * s), ntaps), dim3(256), 0, st, ell, ellz, h, hz,
                       offs_dev, p, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_jacobi_round(double *A, double *V, const int *mdim, const int *ndim, int npad, int ldA,
                        int ldV, int64_t sA, int64_t sV, int batch, int round, double tol,
                        unsigned long long *offmax, hipStream_t st) {
    hipLaunchKernelGGL(jacobi_round, dim3(npad / 2, batch), dim3(256), 0, st, A, V, mdim, ndim,
                       npad, ldA, ldV, sA, sV, round, tol, offmax);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_colnorm(const double *A, const int *mdim, const int *ndim, int ldA, int64_t sA,
                   int npad, int batch, double *sigma, hipStream_t st) {
    hipLaunchKernelGGL(colnorm_kernel, dim3(npad, batch), dim3(256), 0, st, A, mdim, ndim, ldA, sA,
                       npad, sigma);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_svd_gather(const double *A, const double *V, int ldA, int ldV, int m, int n, int k,
                      const int *order, const double *sig, double *UT, double *W, hipStream_t st) {
    hipLaunchKernelGGL(svd_gather, dim3(k), dim3(256), 0, st, A, V, ldA, ldV, m, n, k, order, sig,
                       UT, W);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_gemm_f64(int M, int N, int K, const double *A, int lda, int64_t sA, const double *B,
                    int ldb, int64_t sB, double *C, int ldc, int64_t sC, int batch,
                    hipStream_t st) {
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch);
    hipLaunchKernelGGL(gemm_f64, grid, dim3(256), 0, st, M, N, K, A, lda, sA, B, ldb, sB, C, ldc,
                       sC);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_cast_pad(const double *src, int M, int K, int64_t sS, T *dst, int Mp, int Kp,
                    int64_t sD, int batch, double scale, hipStream_t st) {
    hipLaunchKernelGGL(cast_pad<T>, dim3(blocks_for((int64_t)Mp * Kp), batch), dim3(256), 0, st,
                       src, M, K, sS, dst, Mp, Kp, sD, scale);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int launch_cast_pad_lo(const double *src, int M, int K, int64_t sS, __bf16 *dst, int Mp, int Kp,
                       int64_t sD, int batch, double scale, hipStream_t st) {
    hipLaunchKernelGGL(cast_pad_lo, dim3(blocks_for((int64_t)Mp * Kp), batch), dim3(256), 0, st, src, M,
                       K, sS, dst, Mp, Kp, sD, scale);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template int launch_cast_pad<float>(const double *, int, int, int64_t, float *, int, int, int64_t,
                                    int, double, hipStream_t);
template int launch_cast_pad<double>(const double *, int, int, int64_t, double *, int, int,
                                     int64_t, int, double, hipStream_t);
template int launch_cast_pad<__bf16>(const double *, int, int, int64_t, __bf16 *, int, int,
                                     int64_t, int, double, hipStream_t);
template int launch_cast_pad<_Float16>(const double *, int, int, int64_t, _Float16 *, int, int,
                                       int64_t, int, double, hipStream_t);

}  // namespace kifmm
