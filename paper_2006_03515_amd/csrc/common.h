// Shared definitions of libkifmm (device helpers, error plumbing, internal
// structures).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/kifmm.h"

namespace kifmm {

// ---------------------------------------------------------------- errors ----
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define KIFMM_TRY_(x)                         \
    do {                                      \
        int rc_ = (x);                        \
        if (rc_ != KIFMM_OK) return rc_;      \
    } while (0)

#define KIFMM_HIP(call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------ split BF16 ----
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// FP32 value -> BF16 high part (round to nearest even) and the BF16 of what remains: hi + lo
// holds about 16 of the value's 24 mantissa bits (finite values)
__device__ __forceinline__ void split_bf16(float v, uint16_t &hi, uint16_t &lo) {
    uint32_t u = __float_as_uint(v);
    const uint32_t h = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    hi = (uint16_t)(h >> 16);
    const float r = v - __uint_as_float(h);
    const uint32_t ur = __float_as_uint(r);
    lo = (uint16_t)((ur + 0x7fffu + ((ur >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------ Morton keys ---
// 3D Morton key of box coordinates, bits interleaved ... x1 y1 z1 x0 y0 z0
// (x most significant of each triple).  10 bits per axis.
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}
__host__ __device__ inline uint32_t morton_encode(uint32_t x, uint32_t y, uint32_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
__host__ __device__ inline void morton_decode(uint32_t key, int &x, int &y, int &z) {
    x = (int)compact3(key >> 2);
    y = (int)compact3(key >> 1);
    z = (int)compact3(key);
}

// ------------------------------------------------------------ structures ----
// The tree over the grid: R cubes ("roots") of 2^D x 2^D x 2^D leaves stacked along z, each
// a complete octree.  A leaf holds ell x ell x ellz cells (x, y, z).  A cubic grid of cubic
// cells has R = 1 and ellz = ell; a box nx = ny = ell 2^D, nz = R ellz 2^D with cells of
// hx = hy != hz takes R > 1 and ellz chosen so that leaves are nearly cubic in space.  Boxes
// of level l are numbered root * 8^l + morton(x, y, z - root 2^l), leaves (l = D) likewise,
// so children of box b are 8 b .. 8 b + 7 and its parent b >> 3 as in a single octree.
struct Tree {
    uint64_t magic;       // identifies the tree for ops/tree matching
    int n;                // cells along x and y
    int nz;               // cells along z (n for a cube)
    int ell;              // leaf side in cells along x and y
    int ellz;             // leaf side in cells along z
    int nb;               // leaves per axis of one root cube (2^D)
    int R;                // root cubes along z
    int depth;            // D: levels 0..D, leaves at D
    int s;                // points per leaf = ell^2 ellz
    int64_t N;            // n^2 nz
    double h, hz, x0, y0, z0;   // h = hx = hy
    int32_t *perm;        // device: perm[p] = grid index of leaf-ordered slot p
};

// One "tap GEMM" launch description: for every output box b of a class,
//   out[b][0:M] (+)= sum over taps t of A[op_t] (M x K) * in[src(b, t)][0:K]
enum SrcMode { SRC_SAME = 0, SRC_CHILD = 1, SRC_PARENT = 2, SRC_NBR = 3 };

struct TapList {
    int nclass;        // 1 or 8
    int ntaps;         // taps per class (uniform)
    int *op_dev;       // [nclass][ntaps] operator index
    int *off_dev;      // [nclass][ntaps] packed offset or child index
};

}  // namespace kifmm

struct kifmm_tree_s : kifmm::Tree {};
