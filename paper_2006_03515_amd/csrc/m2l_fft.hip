// M2L in the Fourier domain (the FFT form of eq. (m2l), Section 3 remark).
//
// With the upward equivalent points y^u and the downward check points x^d of a level on
// m0^3 lattices of one spacing t, the M2L matrix of offset o has entries
// G(x^d_i, y^u_j + 2 r o) = g_o(i - j), a block of a 3-D convolution.  On the cyclic grid
// of N = 2 m0 - 1 points per axis the product becomes a pointwise product of spectra:
//     P_t(f) = sum over the interaction list of t:  Gh_o(f) * E_s(f)
// with E_s the half spectrum (N x N x (N+1)/2 complex values) of source box s's
// equivalent density and Gh_o the spectrum of g_o.  The transforms to and from the
// spectra are dense per-box matrices folded into the coefficient bases and run as tap
// GEMMs; this file holds the sums of pointwise products.
//
// For one frequency the sum is a 189-tap stencil over the boxes, with no contraction of its
// own.  Grouped by parents it becomes one: the 8 children c_t of a target parent p take
// products with the 8 children c_s of each of the 27 parents p + d, with the spectrum of
// offset o = 2 d + c_s - c_t (zero where the two children are adjacent).  Written over the
// reals (re, im interleaved), that is a 16 x 432 matrix per frequency applied to 432 gathered
// values per parent: a GEMM with 16 rows, K = 432 and one column per parent.
//
//   m2l_pair_mfma_kernel one workgroup per aligned 4^3 block of parents (512 target boxes) and
//                        4 frequencies; the spectra of the block's source region (6^3
//                        parents x 8 children) are staged in LDS, [frequency][child][re/im]
//                        [parent] so that 16 lanes reading 16 parents hit distinct banks.
//                        Wave w takes frequency w: 4 column blocks of 16 parents on
//                        v_mfma_f32_16x16x4f32, operator fragments read from a table laid out
//                        per frequency as [108 k-steps][64 lanes].  Levels with at least 4
//                        parents per axis.
//   m2l_hadamard_kernel  (levels with fewer parents) one workgroup per aligned 4^3 block
//                        of target boxes (64 consecutive Morton indices) and 16
//                        frequencies, on the FP32 VALU.  The block's
//                        interaction lists lie in the block grown by 2 boxes on every
//                        side (the children of the parents' neighbours), an 8^3 box tile
//                        staged in LDS once and read by all 189 taps.  Wave w takes the
//                        8 targets of class w (the child position, which fixes the tap
//                        list); lane = 16 frequencies x 4 pairs of targets, so every
//                        tap's operator entry is read once per two targets.
#include "common.h"
#include "tapgemm.h"

namespace kifmm {

namespace {

constexpr int HFC = 16;   // frequencies per workgroup

__global__ __launch_bounds__(512) void m2l_hadamard_kernel(const float2 *__restrict__ E, const float2 *__restrict__ Gh,
                                                           const int *__restrict__ tap_op,
                                                           const int *__restrict__ tap_off, int ntaps, int nl,
                                                           int nfp, const uint8_t *__restrict__ out_need,
                                                           const uint8_t *__restrict__ in_nz, float2 *__restrict__ P) {
    __shared__ __align__(16) float2 Es[512 * HFC];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t blk = blockIdx.x;
    const int f0 = blockIdx.y * HFC;
    if (out_need) {   // the same ballot in every wave: all return or none
        if (__ballot(out_need[64 * blk + lane] != 0) == 0) return;
    }
    int bx, by, bz;
    morton_decode((uint32_t)blk, bx, by, bz);
    bx = 4 * bx - 2;
    by = 4 * by - 2;
    bz = 4 * bz - 2;
    // stage the 8^3 source tile: 16 frequencies = 8 float4 per box
    for (int e = tid; e < 512 * 8; e += 512) {
        const int box = e >> 3, part = e & 7;
        const int x = bx + (box >> 6), y = by + ((box >> 3) & 7), z = bz + (box & 7);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x >= 0 && y >= 0 && z >= 0 && x < nl && y < nl && z < nl) {
            const int64_t src = morton_encode(x, y, z);
            if (!in_nz || in_nz[src]) v = ((const float4 *)(E + src * nfp + f0))[part];
        }
        ((float4 *)Es)[e] = v;
    }
    __syncthreads();
    const int c = __builtin_amdgcn_readfirstlane(tid >> 6);   // class of this wave's targets
    const int f = lane & 15, pr = lane >> 4;
    const int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
    int tl[2], tb[2];   // target: Morton index inside the block, and tile index of its box
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int e = 2 * pr + s;
        const int tx = 2 * (e >> 2) + cx, ty = 2 * ((e >> 1) & 1) + cy, tz = 2 * (e & 1) + cz;
        tl[s] = (int)morton_encode(tx, ty, tz);
        tb[s] = ((tx + 2) * 8 + (ty + 2)) * 8 + (tz + 2);
    }
    const int *ops = tap_op + c * ntaps, *offs = tap_off + c * ntaps;
    const float2 *g = Gh + f0 + f;
    float ar0 = 0.f, ai0 = 0.f, ar1 = 0.f, ai1 = 0.f;
#pragma unroll 7
    for (int k = 0; k < ntaps; ++k) {
        const int op = ops[k], pk = offs[k];
        const int delta = ((((pk >> 10) & 31) - 16) * 8 + (((pk >> 5) & 31) - 16)) * 8 + ((pk & 31) - 16);
        const float2 kv = g[(int64_t)op * nfp];
        const float2 e0 = Es[(tb[0] + delta) * HFC + f];
        const float2 e1 = Es[(tb[1] + delta) * HFC + f];
        ar0 = fmaf(kv.x, e0.x, fmaf(-kv.y, e0.y, ar0));
        ai0 = fmaf(kv.x, e0.y, fmaf(kv.y, e0.x, ai0));
        ar1 = fmaf(kv.x, e1.x, fmaf(-kv.y, e1.y, ar1));
        ai1 = fmaf(kv.x, e1.y, fmaf(kv.y, e1.x, ai1));
    }
    P[(64 * blk + tl[0]) * nfp + f0 + f] = make_float2(ar0, ai0);
    P[(64 * blk + tl[1]) * nfp + f0 + f] = make_float2(ar1, ai1);
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int PF = 4;   // frequencies per workgroup of the MFMA kernel (one per wave)

// Am[f][ks][lane]: lane l of k-step ks holds entry (row l % 16, k = 4 ks + l / 16) of the
// 16 x 432 real matrix of frequency f; row = 2 c_t + (re/im), k = 16 d + 2 c_s + (re/im).
__global__ __launch_bounds__(256) void m2l_pair_mfma_kernel(const float2 *__restrict__ E, const float *__restrict__ Am,
                                                            int nl, int nfp, const uint8_t *__restrict__ out_need,
                                                            const uint8_t *__restrict__ in_nz,
                                                            float2 *__restrict__ P) {
    __shared__ float Es[PF * 16 * 216];   // [f][c_s][re/im][region parent], reused for the output
    __shared__ int any_wanted;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int np = nl / 2;
    const int64_t pt = blockIdx.x;        // 64 parents 64 pt .. 64 pt + 63, boxes 512 pt ..
    const int f0 = blockIdx.y * PF;
    if (out_need) {
        if (tid == 0) any_wanted = 0;
        __syncthreads();
        if (out_need[512 * pt + tid] || out_need[512 * pt + 256 + tid]) any_wanted = 1;
        __syncthreads();
        if (!any_wanted) return;
    }
    int ox, oy, oz;
    morton_decode((uint32_t)pt, ox, oy, oz);
    ox = 4 * ox - 1;
    oy = 4 * oy - 1;
    oz = 4 * oz - 1;
    for (int e = tid; e < 216 * 8; e += 256) {
        const int q = e >> 3, c = e & 7;
        const int x = ox + q / 36, y = oy + (q / 6) % 6, z = oz + q % 6;
        float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
        if (x >= 0 && y >= 0 && z >= 0 && x < np && y < np && z < np) {
            const int64_t box = 8 * (int64_t)morton_encode(x, y, z) + c;
            if (!in_nz || in_nz[box]) {
                const float4 *src = (const float4 *)(E + box * nfp + f0);
                v0 = src[0];
                v1 = src[1];
            }
        }
        Es[((0 * 8 + c) * 2 + 0) * 216 + q] = v0.x;
        Es[((0 * 8 + c) * 2 + 1) * 216 + q] = v0.y;
        Es[((1 * 8 + c) * 2 + 0) * 216 + q] = v0.z;
        Es[((1 * 8 + c) * 2 + 1) * 216 + q] = v0.w;
        Es[((2 * 8 + c) * 2 + 0) * 216 + q] = v1.x;
        Es[((2 * 8 + c) * 2 + 1) * 216 + q] = v1.y;
        Es[((3 * 8 + c) * 2 + 0) * 216 + q] = v1.z;
        Es[((3 * 8 + c) * 2 + 1) * 216 + q] = v1.w;
    }
    __syncthreads();
    // lane: k slot g = lane / 16 of each MFMA, parent 16 nb + lane % 16 of column block nb
    const int g = lane >> 4;
    int qn[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        int a, b, c;
        morton_decode((uint32_t)(16 * nb + (lane & 15)), a, b, c);
        qn[nb] = ((a + 1) * 6 + (b + 1)) * 6 + (c + 1);
    }
    floatx4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float *Af = Am + (int64_t)(f0 + w) * 108 * 64 + lane;
    const float *Ew = Es + w * 16 * 216 + g * 216;
    for (int d = 0; d < 27; ++d) {   // source parent p + (dx, dy, dz), d = 9 (dx+1) + 3 (dy+1) + dz+1
        const int dq = ((d / 9 - 1) * 6 + ((d / 3) % 3 - 1)) * 6 + (d % 3 - 1);
        float a4[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a4[s] = Af[(4 * d + s) * 64];
#pragma unroll
        for (int s = 0; s < 4; ++s) {   // k-step 4 d + s: c_s = 2 s + g / 2, re/im = g % 2
            const float *eb = Ew + s * 4 * 216 + dq;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[s], eb[qn[nb]], acc[nb], 0, 0, 0);
        }
    }
    __syncthreads();
    // D layout of 16x16x4: lane holds rows 4 g + v of column lane % 16; row = 2 c_t + re/im
    float *Os = Es;   // [parent][c_t][f][re/im] = the 512 target boxes' 4 frequencies, in order
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int n = 16 * nb + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * g + v;
            Os[((n * 8 + (row >> 1)) * PF + w) * 2 + (row & 1)] = acc[nb][v];
        }
    }
    __syncthreads();
    for (int e = tid; e < 512 * 2; e += 256) {
        const int bl = e >> 1, half = e & 1;
        ((float4 *)(P + (512 * pt + bl) * nfp + f0))[half] = ((const float4 *)Os)[bl * 2 + half];
    }
}

}  // namespace

int run_m2l_pair_mfma(const float *E, const float *Am, int nl, int nfp, const uint8_t *out_need,
                      const uint8_t *in_nz, float *P, hipStream_t st) {
    if (nl < 8 || (nl & (nl - 1)) != 0) return fail(KIFMM_EINVAL, "M2L spectra: boxes per axis must be 8, 16, ...");
    if (nfp % PF != 0) return fail(KIFMM_EINVAL, "M2L spectra: frequency count not a multiple of 4");
    const int64_t ntile = (int64_t)nl * nl * nl / 512;
    hipLaunchKernelGGL(m2l_pair_mfma_kernel, dim3((unsigned)ntile, (unsigned)(nfp / PF)), dim3(256), 0, st,
                       (const float2 *)E, Am, nl, nfp, out_need, in_nz, (float2 *)P);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_m2l_hadamard(const float *E, const float *Gh, const int *tap_op, const int *tap_off, int ntaps, int nl,
                     int nfp, const uint8_t *out_need, const uint8_t *in_nz, float *P, hipStream_t st) {
    if (nl < 4 || (nl & (nl - 1)) != 0) return fail(KIFMM_EINVAL, "M2L spectra: boxes per axis must be 4, 8, 16, ...");
    if (nfp % HFC != 0) return fail(KIFMM_EINVAL, "M2L spectra: frequency count not a multiple of 16");
    const int64_t nblk = (int64_t)nl * nl * nl / 64;
    hipLaunchKernelGGL(m2l_hadamard_kernel, dim3((unsigned)nblk, (unsigned)(nfp / HFC)), dim3(512), 0, st,
                       (const float2 *)E, (const float2 *)Gh, tap_op, tap_off, ntaps, nl, nfp, out_need, in_nz,
                       (float2 *)P);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
