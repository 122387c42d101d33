// Octree over a uniform grid (Section 3, tree construction step).
//
// The complete octree with ell x ell x ellz-cell leaves (one per root cube; a box grid
// is a column of R root cubes along z) is visited in pre-order by the Morton order of
// the leaves, root after root.  Every cell gets the key
//     key = (root * nb^3 + morton(leaf coordinates in its root)) * s
//           + (C-order index inside the leaf),   s = ell^2 ellz
// Keys are distinct and cover [0, N) exactly, so sorting the cells by key is a
// single scatter perm[key] = cell (a counting sort whose buckets hold one cell
// each).  perm is kept for callers; the evaluation's permutes recompute
// cell = perm[p] from p by decoding the key instead of reading perm.
#include "common.h"

namespace kifmm {

namespace {

// Shape of the leaf order (all sides powers of two): lg of ell, ellz, nb; n, nz
struct Shape {
    int n, nz, lg_ell, lg_ellz, lg_nb;
};

Shape shape_of(const Tree &t) {
    auto lg = [](int v) { int l = 0; while ((1 << l) < v) ++l; return l; };
    return Shape{t.n, t.nz, lg(t.ell), lg(t.ellz), lg(t.nb)};
}

// leaf-ordered slot of grid cell (i, j, k)
__device__ inline int64_t slot_of_cell(int i, int j, int k, const Shape &sh) {
    const int lz_all = k >> sh.lg_ellz;                       // leaf z in the column
    const int root = lz_all >> sh.lg_nb, lz = lz_all & ((1 << sh.lg_nb) - 1);
    const int64_t leaf = ((int64_t)root << (3 * sh.lg_nb)) + morton_encode(i >> sh.lg_ell, j >> sh.lg_ell, lz);
    const int mx = (1 << sh.lg_ell) - 1, mz = (1 << sh.lg_ellz) - 1;
    const int64_t local = ((int64_t)(i & mx) << (sh.lg_ell + sh.lg_ellz)) + ((j & mx) << sh.lg_ellz) + (k & mz);
    return (leaf << (2 * sh.lg_ell + sh.lg_ellz)) + local;
}

__global__ void morton_scatter_kernel(Shape sh, int64_t N, int32_t *perm) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(g / ((int64_t)sh.n * sh.nz));
        const int j = (int)((g / sh.nz) % sh.n);
        const int k = (int)(g % sh.nz);
        perm[slot_of_cell(i, j, k, sh)] = (int32_t)g;
    }
}

// Grid index of leaf-ordered slot p (the inverse of slot_of_cell): p = leaf * s + local,
// leaf = root * nb^3 + a Morton code of leaf coordinates in the root, local the C-order
// index inside the leaf.
__device__ inline int64_t cell_of_slot(int64_t p, const Shape &sh) {
    const int lg_s = 2 * sh.lg_ell + sh.lg_ellz;
    const int64_t leaf = p >> lg_s;
    const int local = (int)(p & ((1 << lg_s) - 1));
    const int64_t root = leaf >> (3 * sh.lg_nb);
    int lx, ly, lz;
    morton_decode((uint32_t)(leaf & ((1ll << (3 * sh.lg_nb)) - 1)), lx, ly, lz);
    const int i = (lx << sh.lg_ell) | (local >> (sh.lg_ell + sh.lg_ellz));
    const int j = (ly << sh.lg_ell) | ((local >> sh.lg_ellz) & ((1 << sh.lg_ell) - 1));
    const int64_t k = (((root << sh.lg_nb) + lz) << sh.lg_ellz) | (local & ((1 << sh.lg_ellz) - 1));
    return ((int64_t)i * sh.n + j) * sh.nz + k;
}

// q[p] = scale * I[cell(p)] (FP32 or FP64 in, same type out)
template <typename T>
__global__ void permute_in_kernel(const T *__restrict__ I, Shape sh, int64_t N, T scale, T *__restrict__ q) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x)
        q[p] = I[cell_of_slot(p, sh)] * scale;
}

// S[cell(p)] = scale * Sp[p], or 0 where want (one byte per leaf, leaf order; null: every
// leaf is wanted) marks the leaf of slot p as not wanted
template <typename T>
__global__ void permute_out_kernel(const T *__restrict__ Sp, Shape sh, int64_t N, T scale,
                                   const uint8_t *__restrict__ want, T *__restrict__ S) {
    const int lg_s = 2 * sh.lg_ell + sh.lg_ellz;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        T v = 0;
        if (!want || want[p >> lg_s]) v = Sp[p] * scale;
        S[cell_of_slot(p, sh)] = v;
    }
}

// S[cell(p)] = scale * (Sa[p] + Sb[p])  (far field + near field), 0 where not wanted
template <typename T>
__global__ void permute_out2_kernel(const T *__restrict__ Sa, const T *__restrict__ Sb, Shape sh,
                                    int64_t N, T scale, const uint8_t *__restrict__ want, T *__restrict__ S) {
    const int lg_s = 2 * sh.lg_ell + sh.lg_ellz;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        T v = 0;
        if (!want || want[p >> lg_s]) v = (Sa[p] + Sb[p]) * scale;
        S[cell_of_slot(p, sh)] = v;
    }
}

// Leaves of 8^3 cells on a grid with n a multiple of 32: one thread per run of 32 cells along
// k of a grid row (i, j), 128 contiguous bytes on the grid side; on the leaf side the run is
// the 8-cell lines (i & 7, j & 7) of 4 leaves, 32 contiguous bytes each.  Thread order
// t = (i n + j) (n / 32) + k / 32.
__device__ inline void row_of_thread(int64_t t, int n, int &i, int &j, int &kb) {
    const int nk = n >> 5;
    kb = (int)(t % nk);
    const int64_t ij = t / nk;
    j = (int)(ij % n);
    i = (int)(ij / n);
}

__global__ __launch_bounds__(256) void permute_in_rows_kernel(const float *__restrict__ I, int n, int64_t nrows,
                                                              float scale, float *__restrict__ q) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nrows) return;
    int i, j, kb;
    row_of_thread(t, n, i, j, kb);
    const float4 *src = (const float4 *)(I + ((int64_t)i * n + j) * n + 32 * kb);
    const int local = ((i & 7) * 8 + (j & 7)) * 8;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 a = src[2 * c], b = src[2 * c + 1];
        float4 *dst = (float4 *)(q + (int64_t)morton_encode(i >> 3, j >> 3, 4 * kb + c) * 512 + local);
        dst[0] = make_float4(a.x * scale, a.y * scale, a.z * scale, a.w * scale);
        dst[1] = make_float4(b.x * scale, b.y * scale, b.z * scale, b.w * scale);
    }
}

// Leaves of 8^3 cells: one thread per 8-cell line (i & 7, j & 7) of a leaf, read contiguous
// in leaf order (a wave reads 2 KB in one piece) and written as 32 contiguous bytes of grid
// row (i, j).
__global__ __launch_bounds__(256) void permute_out2_lines_kernel(const float *__restrict__ Sa, const float *__restrict__ Sb,
                                                                 int n, int64_t nlines, float scale,
                                                                 const uint8_t *__restrict__ want, float *__restrict__ S) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nlines) return;
    const uint32_t leaf = (uint32_t)(t >> 6);
    const int line = (int)(t & 63);
    int lx, ly, lz;
    morton_decode(leaf, lx, ly, lz);
    const int i = (lx << 3) | (line >> 3), j = (ly << 3) | (line & 7);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    if (!want || want[leaf]) {
        const float4 a0 = ((const float4 *)Sa)[2 * t], a1 = ((const float4 *)Sa)[2 * t + 1];
        const float4 b0 = ((const float4 *)Sb)[2 * t], b1 = ((const float4 *)Sb)[2 * t + 1];
        a = make_float4((a0.x + b0.x) * scale, (a0.y + b0.y) * scale, (a0.z + b0.z) * scale, (a0.w + b0.w) * scale);
        b = make_float4((a1.x + b1.x) * scale, (a1.y + b1.y) * scale, (a1.z + b1.z) * scale, (a1.w + b1.w) * scale);
    }
    float4 *dst = (float4 *)(S + ((int64_t)i * n + j) * n + (lz << 3));
    dst[0] = a;
    dst[1] = b;
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
    hipLaunchKernelGGL(morton_scatter_kernel, dim3(grid_for(t.N)), dim3(256), 0, st, shape_of(t), t.N, t.perm);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_in(const Tree &t, const T *I, T scale, T *q, hipStream_t st) {
    if (sizeof(T) == 4 && t.ell == 8 && t.ellz == 8 && t.R == 1 && t.n % 32 == 0 && (uintptr_t)I % 16 == 0) {   // whole 128-byte rows
        const int64_t nrows = t.N / 32;
        hipLaunchKernelGGL(permute_in_rows_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st,
                           (const float *)I, t.n, nrows, (float)scale, (float *)q);
        KIFMM_HIP(hipGetLastError());
        return KIFMM_OK;
    }
    hipLaunchKernelGGL(permute_in_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, I, shape_of(t), t.N, scale, q);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_out(const Tree &t, const T *Sp, T scale, const uint8_t *want, T *S, hipStream_t st) {
    hipLaunchKernelGGL(permute_out_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, Sp, shape_of(t), t.N, scale,
                       want, S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename T>
int launch_permute_out2(const Tree &t, const T *Sa, const T *Sb, T scale, const uint8_t *want, T *S,
                        hipStream_t st) {
    if (sizeof(T) == 4 && t.ell == 8 && t.ellz == 8 && t.R == 1 && (uintptr_t)S % 16 == 0) {   // whole 8-cell lines
        const int64_t nlines = t.N / 8;
        hipLaunchKernelGGL(permute_out2_lines_kernel, dim3((unsigned)((nlines + 255) / 256)), dim3(256), 0, st,
                           (const float *)Sa, (const float *)Sb, t.n, nlines, (float)scale, want, (float *)S);
        KIFMM_HIP(hipGetLastError());
        return KIFMM_OK;
    }
    hipLaunchKernelGGL(permute_out2_kernel<T>, dim3(grid_for(t.N)), dim3(256), 0, st, Sa, Sb, shape_of(t), t.N,
                       scale, want, S);
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
