// Octree over a uniform n^3 grid (Section 3, tree construction step).
//
// The complete octree with ell^3-cell leaves is visited in pre-order by the
// Morton order of the leaves.  Every cell gets the key
//     key = morton(leaf coordinates) * ell^3 + (C-order index inside the leaf)
// Keys are distinct and cover [0, N) exactly, so sorting the cells by key is a
// single scatter perm[key] = cell (a counting sort whose buckets hold one cell
// each).  perm is kept for callers; the evaluation's permutes recompute
// cell = perm[p] from p by decoding the key instead of reading perm.
#include "common.h"

namespace kifmm {

namespace {

__global__ void morton_scatter_kernel(int n, int ell, int lg_ell, int64_t N, int32_t *perm) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(g / ((int64_t)n * n));
        const int j = (int)((g / n) % n);
        const int k = (int)(g % n);
        const uint32_t leaf = morton_encode(i >> lg_ell, j >> lg_ell, k >> lg_ell);
        const int mask = ell - 1;
        const int64_t local = (((int64_t)(i & mask) * ell) + (j & mask)) * ell + (k & mask);
        const int64_t key = (int64_t)leaf * ((int64_t)ell * ell * ell) + local;
        perm[key] = (int32_t)g;
    }
}

// Grid index of leaf-ordered slot p (the inverse of the key above): p = leaf * ell^3 +
// local, leaf a Morton code of leaf coordinates, local the C-order index inside it.
__device__ inline int64_t cell_of_slot(int64_t p, int n, int lg_ell) {
    const int lg_s = 3 * lg_ell, mask = (1 << lg_ell) - 1;
    const uint32_t leaf = (uint32_t)(p >> lg_s);
    const int local = (int)(p & ((1 << lg_s) - 1));
    int lx, ly, lz;
    morton_decode(leaf, lx, ly, lz);
    const int i = (lx << lg_ell) | (local >> (2 * lg_ell));
    const int j = (ly << lg_ell) | ((local >> lg_ell) & mask);
    const int k = (lz << lg_ell) | (local & mask);
    return ((int64_t)i * n + j) * n + k;
}

// q[p] = scale * I[cell(p)] (FP32 or FP64 in, same type out)
template <typename T>
__global__ void permute_in_kernel(const T *__restrict__ I, int n, int lg_ell, int64_t N, T scale, T *__restrict__ q) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x)
        q[p] = I[cell_of_slot(p, n, lg_ell)] * scale;
}

// S[cell(p)] = scale * Sp[p], or 0 where want (one byte per leaf, Morton order; null: every
// leaf is wanted) marks the leaf of slot p as not wanted
template <typename T>
__global__ void permute_out_kernel(const T *__restrict__ Sp, int n, int lg_ell, int64_t N, T scale,
                                   const uint8_t *__restrict__ want, T *__restrict__ S) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        T v = 0;
        if (!want || want[p >> (3 * lg_ell)]) v = Sp[p] * scale;
        S[cell_of_slot(p, n, lg_ell)] = v;
    }
}

// S[cell(p)] = scale * (Sa[p] + Sb[p])  (far field + near field), 0 where not wanted
template <typename T>
__global__ void permute_out2_kernel(const T *__restrict__ Sa, const T *__restrict__ Sb, int n, int lg_ell,
                                    int64_t N, T scale, const uint8_t *__restrict__ want, T *__restrict__ S) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        T v = 0;
        if (!want || want[p >> (3 * lg_ell)]) v = (Sa[p] + Sb[p]) * scale;
        S[cell_of_slot(p, n, lg_ell)] = v;
    }
}

__global__ void perm_to_i64_kernel(const int32_t *perm, int64_t N, int64_t *out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p] = perm[p];
}

int lg_of(int ell) {
    int lg = 0;
    while ((1 << lg) < ell) ++lg;
    return lg;
}

unsigned grid_for(int64_t N) {
    int64_t b = (N + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

int launch_morton_scatter(const Tree &t, hipStream_t st) {
    hipLaunchKernelGGL(morton_scatter_kernel, dim3(grid_for(t.N)), dim3(256), 0, st, t.n, t.ell,
                       lg_of(t.ell), t.N, t.perm);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_in(const Tree &t, const T *I, T scale, T *q, hipStream_t st) {
    hipLaunchKernelGGL(permute_in_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, I, t.n, lg_of(t.ell),
                       t.N, scale, q);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_out(const Tree &t, const T *Sp, T scale, const uint8_t *want, T *S, hipStream_t st) {
    hipLaunchKernelGGL(permute_out_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, Sp, t.n, lg_of(t.ell),
                       t.N, scale, want, S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_out2(const Tree &t, const T *Sa, const T *Sb, T scale, const uint8_t *want, T *S,
                        hipStream_t st) {
    hipLaunchKernelGGL(permute_out2_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, Sa, Sb, t.n,
                       lg_of(t.ell), t.N, scale, want, S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}
template int launch_permute_out2<float>(const Tree &, const float *, const float *, float, const uint8_t *,
                                        float *, hipStream_t);
template int launch_permute_out2<double>(const Tree &, const double *, const double *, double,
                                         const uint8_t *, double *, hipStream_t);

int launch_perm_i64(const Tree &t, int64_t *out, hipStream_t st) {
    hipLaunchKernelGGL(perm_to_i64_kernel, dim3(grid_for(t.N)), dim3(256), 0, st, t.perm, t.N,
                       out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template int launch_permute_in<float>(const Tree &, const float *, float, float *, hipStream_t);
template int launch_permute_in<double>(const Tree &, const double *, double, double *, hipStream_t);
template int launch_permute_out<float>(const Tree &, const float *, float, const uint8_t *, float *,
                                       hipStream_t);
template int launch_permute_out<double>(const Tree &, const double *, double, const uint8_t *, double *,
                                        hipStream_t);

}  // namespace kifmm
