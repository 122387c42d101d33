// M2L in the Fourier domain (the FFT form of eq. (m2l), Section 3 remark).
//
// With the upward equivalent points y^u and the downward check points x^d of a level on
// m0^3 lattices of one spacing t, the M2L matrix of offset o has entries
// G(x^d_i, y^u_j + 2 r o) = g_o(i - j), a block of a 3-D convolution.  On the cyclic grid
// of N = 2 m0 - 1 points per axis the product becomes a pointwise product of spectra:
//     P_t(f) = sum over the interaction list of t:  Gh_o(f) * E_s(f)
// with E_s the spectrum of source box s's equivalent density at (N^3 + 1)/2 frequencies (one
// of each conjugate pair: the density is real) and Gh_o the spectrum of g_o.  Coefficients
// become lattice values through the bases (tap GEMMs, W_u and U_d^T); this file holds the
// separable transforms
// between lattice values and spectra, and the sums of pointwise products.
//
// For one frequency the sum is a 189-tap stencil over the boxes, with no contraction of its
// own.  Grouped by parents it becomes one: the 8 children c_t of a target parent p take
// products with the 8 children c_s of each of the 27 parents p + d, with the spectrum of
// offset o = 2 d + c_s - c_t (zero where the two children are adjacent).  Written over the
// reals (re, im interleaved), that is a 16 x 432 matrix per frequency applied to 432 gathered
// values per parent: a GEMM with 16 rows, K = 432 and one column per parent.
//
//   m2l_lattice_forward_kernel / m2l_lattice_inverse_kernel  one wave per box: the
//                        separable transforms between the m0^3 lattice values and the half
//                        spectrum (z, y, x stages; inverse x, y, z).
//   m2l_pair_mfma_kernel one workgroup per aligned 4^3 block of parents (512 target boxes) and
//                        4 frequencies; the spectra of the block's source region (6^3
//                        parents x 8 children) are staged in LDS, [frequency][parent][k slot]
//                        [k-step], so that one 16-byte read gives a lane the four k-steps of
//                        one source parent that its four MFMAs take in turn.
//                        Wave w takes frequency w: 4 column blocks of 16 parents on
//                        v_mfma_f32_16x16x4f32, operator fragments read from a table laid out
//                        per frequency as [27 parents][64 lanes][4 k-steps].  Levels with at least 4
//                        parents per axis.
//   m2l_pair_bf16x3_kernel the same in split BF16 on v_mfma_f32_16x16x32_bf16 (precision
//                        KIFMM_BF16X3).
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

// Workgroup -> (block of 4^3 parents, frequency group).  Workgroups are dealt to the 8 XCDs
// in turn; when the blocks divide by 8, XCD x takes the blocks x B/8 .. (x+1) B/8 - 1 (a
// Morton-contiguous region) for one frequency group after another, so the halos that
// neighbouring blocks share are read from that XCD's L2 instead of once per block.
__device__ __forceinline__ void pair_tile(int64_t &pt, int &fg) {
    const int nb = gridDim.x;
    if ((nb & 7) == 0) {
        const int64_t i = blockIdx.x + (int64_t)nb * blockIdx.y;
        const int per = nb >> 3;
        const int64_t j = i >> 3;
        pt = (int64_t)(i & 7) * per + j % per;
        fg = (int)(j / per);
    } else {
        pt = blockIdx.x;
        fg = blockIdx.y;
    }
}

// Am[f][d][lane][s]: lane l of k-step ks = 4 d + s holds entry (row l % 16, k = 4 ks + l / 16)
// of the 16 x 432 real matrix of frequency f; row = 2 c_t + (re/im), k = 16 d + 2 c_s + (re/im).
__global__ __launch_bounds__(256) void m2l_pair_mfma_kernel(const float2 *__restrict__ E, const float *__restrict__ Am,
                                                            int nl, int nfp, const uint8_t *__restrict__ out_need,
                                                            const uint8_t *__restrict__ in_nz,
                                                            float2 *__restrict__ P) {
    __shared__ __align__(16) float Es[PF * 16 * 216];   // [f][region parent][k slot][k-step], reused for the output
    __shared__ int any_wanted;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int np = nl / 2;
    int64_t pt;                           // 64 parents 64 pt .. 64 pt + 63, boxes 512 pt ..
    int fg;
    pair_tile(pt, fg);
    const int f0 = fg * PF;
    if (out_need) {
        if (tid == 0) any_wanted = 0;
        __syncthreads();
        if (out_need[512 * pt + tid] || out_need[512 * pt + 256 + tid]) any_wanted = 1;
        __syncthreads();
        if (!any_wanted) return;
    }
    // this wave's operator fragments (26 source parents x 4 k-steps) and the workgroup's share
    // of the source region's spectra are requested together, before anything waits: one
    // memory latency per workgroup instead of one per staging round and per source parent
    const float4 *Af = (const float4 *)(Am + (int64_t)(f0 + w) * 108 * 64) + lane;
    float4 a[26];
#pragma unroll
    for (int d = 0; d < 27; ++d)
        if (d != 13) a[d - (d > 13)] = Af[d * 64];
    int ox, oy, oz;
    morton_decode((uint32_t)pt, ox, oy, oz);
    ox = 4 * ox - 1;
    oy = 4 * oy - 1;
    oz = 4 * oz - 1;
    constexpr int NST = (216 * 8 + 255) / 256;   // staging rounds: 216 parents x 8 children
    float4 v[NST][2];
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        const int x = ox + q / 36, y = oy + (q / 6) % 6, z = oz + q % 6;
        v[i][0] = v[i][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < 216 * 8 && x >= 0 && y >= 0 && z >= 0 && x < np && y < np && z < np) {
            const int64_t box = 8 * (int64_t)morton_encode(x, y, z) + c;
            if (!in_nz || in_nz[box]) {
                const float4 *src = (const float4 *)(E + box * nfp + f0);
                v[i][0] = src[0];
                v[i][1] = src[1];
            }
        }
    }
    // LDS layout [f][region parent][k slot g][k-step s]: row 2 c_s + re/im = 4 s + g of the
    // operator, so a lane's four k-steps of one source parent are one 16-byte read
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        if (e < 216 * 8) {
            const int gs = 4 * (2 * (c & 1)) + (c >> 1);   // (g, s) of re; im is g + 1
            Es[((0 * 216 + q) * 4) * 4 + gs] = v[i][0].x;
            Es[((0 * 216 + q) * 4) * 4 + gs + 4] = v[i][0].y;
            Es[((1 * 216 + q) * 4) * 4 + gs] = v[i][0].z;
            Es[((1 * 216 + q) * 4) * 4 + gs + 4] = v[i][0].w;
            Es[((2 * 216 + q) * 4) * 4 + gs] = v[i][1].x;
            Es[((2 * 216 + q) * 4) * 4 + gs + 4] = v[i][1].y;
            Es[((3 * 216 + q) * 4) * 4 + gs] = v[i][1].z;
            Es[((3 * 216 + q) * 4) * 4 + gs + 4] = v[i][1].w;
        }
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
    const floatx4 *Ew = (const floatx4 *)Es + w * 216 * 4 + g;   // [q][g]: the 4 k-steps
#pragma unroll
    for (int d = 0; d < 27; ++d) {   // source parent p + (dx, dy, dz), d = 9 (dx+1) + 3 (dy+1) + dz+1
        if (d == 13) continue;   // the target's own parent: all its children are adjacent (zeros)
        const int dq = ((d / 9 - 1) * 6 + ((d / 3) % 3 - 1)) * 6 + (d % 3 - 1);
        const float4 ad = a[d - (d > 13)];   // k-steps 4 d .. 4 d + 3
        const float a4[4] = {ad.x, ad.y, ad.z, ad.w};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            // k-step 4 d + s: c_s = 2 s + g / 2, re/im = g % 2 (the same order of products
            // into each column block's sums as one k-step after the other)
            const floatx4 b = Ew[(qn[nb] + dq) * 4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[s], b[s], acc[nb], 0, 0, 0);
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

// The parent-pair products in split BF16 (A_hi B_hi + A_hi B_lo + A_lo B_hi, FP32
// accumulation, about 16 mantissa bits) on v_mfma_f32_16x16x32_bf16: the same workgroup
// shape as m2l_pair_mfma_kernel, spectra staged as BF16 pairs [f][region parent][c_s][re/im]
// (16 values per parent, hi and lo planes), K = 432 padded to 448 (14 k-steps).  Lane group
// g = lane / 16 of k-step ks reads the 8 values of the source parent at position 2 ks + g / 2
// (13 and 26 swapped), children 4 (g % 2) .. + 3.
__global__ __launch_bounds__(256) void m2l_pair_bf16x3_kernel(const float2 *__restrict__ E, const uint16_t *__restrict__ Ab,
                                                              int nl, int nfp, const uint8_t *__restrict__ out_need,
                                                              const uint8_t *__restrict__ in_nz,
                                                              float2 *__restrict__ P) {
    __shared__ __align__(16) uint16_t Eh[PF * 216 * 16], El[PF * 216 * 16];
    __shared__ int any_wanted;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int np = nl / 2;
    int64_t pt;
    int fg;
    pair_tile(pt, fg);
    const int f0 = fg * PF;
    if (out_need) {
        if (tid == 0) any_wanted = 0;
        __syncthreads();
        if (out_need[512 * pt + tid] || out_need[512 * pt + 256 + tid]) any_wanted = 1;
        __syncthreads();
        if (!any_wanted) return;
    }
    // operator fragments and the source region's spectra requested together (one memory
    // latency per workgroup)
    const uint4 *Af = (const uint4 *)(Ab + ((int64_t)(f0 + w) * 14 * 64 + lane) * 16);
    uint4 ah[13], al[13];
#pragma unroll
    for (int ks = 0; ks < 13; ++ks) {
        ah[ks] = Af[ks * 64 * 2];
        al[ks] = Af[ks * 64 * 2 + 1];
    }
    int ox, oy, oz;
    morton_decode((uint32_t)pt, ox, oy, oz);
    ox = 4 * ox - 1;
    oy = 4 * oy - 1;
    oz = 4 * oz - 1;
    constexpr int NST = (216 * 8 + 255) / 256;
    float4 v[NST][2];
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        const int x = ox + q / 36, y = oy + (q / 6) % 6, z = oz + q % 6;
        v[i][0] = v[i][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < 216 * 8 && x >= 0 && y >= 0 && z >= 0 && x < np && y < np && z < np) {
            const int64_t box = 8 * (int64_t)morton_encode(x, y, z) + c;
            if (!in_nz || in_nz[box]) {
                const float4 *src = (const float4 *)(E + box * nfp + f0);
                v[i][0] = src[0];
                v[i][1] = src[1];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        if (e >= 216 * 8) continue;
        const float vals[8] = {v[i][0].x, v[i][0].y, v[i][0].z, v[i][0].w,
                               v[i][1].x, v[i][1].y, v[i][1].z, v[i][1].w};   // (f, re/im)
#pragma unroll
        for (int f = 0; f < PF; ++f) {
            uint16_t hr, lr, hi, li;
            split_bf16(vals[2 * f], hr, lr);
            split_bf16(vals[2 * f + 1], hi, li);
            const int at = ((f * 216 + q) * 16 + 2 * c) >> 1;   // a (re, im) pair as one 32-bit word
            ((uint32_t *)Eh)[at] = (uint32_t)hr | ((uint32_t)hi << 16);
            ((uint32_t *)El)[at] = (uint32_t)lr | ((uint32_t)li << 16);
        }
    }
    __syncthreads();
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
    const uint16_t *Ehw = Eh + w * 216 * 16 + 8 * (g & 1), *Elw = El + w * 216 * 16 + 8 * (g & 1);
    // k order: position q = 2 ks + g / 2 holds source parent d = q with 13 and 26 swapped, so
    // the last k-step (d = 13, the target's own parent, whose children are all adjacent, and
    // the padding) is all zeros and is skipped
#pragma unroll
    for (int ks = 0; ks < 13; ++ks) {
        const int q = 2 * ks + (g >> 1), d = q == 13 ? 26 : (q == 26 ? 13 : q);
        const int dq = ((d / 9 - 1) * 6 + ((d / 3) % 3 - 1)) * 6 + (d % 3 - 1);
        bf16x8 a_hi, a_lo;
        __builtin_memcpy(&a_hi, &ah[ks], 16);
        __builtin_memcpy(&a_lo, &al[ks], 16);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int q = qn[nb] + dq;
            bf16x8 b_hi, b_lo;
            __builtin_memcpy(&b_hi, Ehw + q * 16, 16);
            __builtin_memcpy(&b_lo, Elw + q * 16, 16);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_hi, acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_lo, acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, b_hi, acc[nb], 0, 0, 0);
        }
    }
    __syncthreads();
    float *Os = (float *)Eh;   // [parent][c_t][f][re/im]: 512 boxes x PF frequencies (16 KB)
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

// The parent-pair products with single FP16 or BF16 operands (FP32 accumulation) on
// v_mfma_f32_16x16x32_{f16,bf16}: the workgroup shape and k order of m2l_pair_bf16x3_kernel,
// one part instead of three.  Operands are scaled by powers of two so that FP16's range holds
// them (and the scaling is exact): each frequency's operator fragments were scaled at the
// precompute (so that its largest entry lies in [2^13, 2^14); `unscale` holds the inverse
// factors), and each workgroup scales the spectra it stages by 2^(14 - e), e the exponent of
// their largest magnitude.  The products are multiplied back in FP32.
template <typename LT>
__device__ __forceinline__ floatx4 mfma_lp32(const LT *a, const LT *b, floatx4 c);
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <>
__device__ __forceinline__ floatx4 mfma_lp32<_Float16>(const _Float16 *a, const _Float16 *b, floatx4 c) {
    f16x8 x, y;
    __builtin_memcpy(&x, a, 16);
    __builtin_memcpy(&y, b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx4 mfma_lp32<__bf16>(const __bf16 *a, const __bf16 *b, floatx4 c) {
    bf16x8 x, y;
    __builtin_memcpy(&x, a, 16);
    __builtin_memcpy(&y, b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

template <typename LT>
__global__ __launch_bounds__(256) void m2l_pair_lp1_kernel(const float2 *__restrict__ E, const LT *__restrict__ Al,
                                                           const float *__restrict__ unscale, int nl, int nfp,
                                                           const uint8_t *__restrict__ out_need,
                                                           const uint8_t *__restrict__ in_nz,
                                                           float2 *__restrict__ P) {
    __shared__ __align__(16) LT Eh[PF * 216 * 16];   // [f][region parent][c_s][re/im], reused for the output
    __shared__ float wmax[4];
    __shared__ int any_wanted;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int np = nl / 2;
    int64_t pt;
    int fg;
    pair_tile(pt, fg);
    const int f0 = fg * PF;
    if (out_need) {
        if (tid == 0) any_wanted = 0;
        __syncthreads();
        if (out_need[512 * pt + tid] || out_need[512 * pt + 256 + tid]) any_wanted = 1;
        __syncthreads();
        if (!any_wanted) return;
    }
    const uint4 *Af = (const uint4 *)(Al + ((int64_t)(f0 + w) * 14 * 64 + lane) * 8);
    uint4 a[13];
#pragma unroll
    for (int ks = 0; ks < 13; ++ks) a[ks] = Af[ks * 64];
    int ox, oy, oz;
    morton_decode((uint32_t)pt, ox, oy, oz);
    ox = 4 * ox - 1;
    oy = 4 * oy - 1;
    oz = 4 * oz - 1;
    constexpr int NST = (216 * 8 + 255) / 256;
    float4 v[NST][2];
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        const int x = ox + q / 36, y = oy + (q / 6) % 6, z = oz + q % 6;
        v[i][0] = v[i][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < 216 * 8 && x >= 0 && y >= 0 && z >= 0 && x < np && y < np && z < np) {
            const int64_t box = 8 * (int64_t)morton_encode(x, y, z) + c;
            if (!in_nz || in_nz[box]) {
                const float4 *src = (const float4 *)(E + box * nfp + f0);
                v[i][0] = src[0];
                v[i][1] = src[1];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NST; ++i)
        m = fmaxf(m, fmaxf(fmaxf(fmaxf(fabsf(v[i][0].x), fabsf(v[i][0].y)), fmaxf(fabsf(v[i][0].z), fabsf(v[i][0].w))),
                           fmaxf(fmaxf(fabsf(v[i][1].x), fabsf(v[i][1].y)), fmaxf(fabsf(v[i][1].z), fabsf(v[i][1].w)))));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) wmax[w] = m;
    __syncthreads();
    m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    int ex = 0;
    if (m > 0.f) frexpf(m, &ex);   // m < 2^ex
    const int sh = min(14 - ex, 126);
    const float scale = ldexpf(1.f, sh), back = ldexpf(1.f, -sh);
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = tid + 256 * i, q = e >> 3, c = e & 7;
        if (e >= 216 * 8) continue;
        const float vals[8] = {v[i][0].x, v[i][0].y, v[i][0].z, v[i][0].w,
                               v[i][1].x, v[i][1].y, v[i][1].z, v[i][1].w};   // (f, re/im)
#pragma unroll
        for (int f = 0; f < PF; ++f) {
            LT pr[2] = {(LT)(vals[2 * f] * scale), (LT)(vals[2 * f + 1] * scale)};
            __builtin_memcpy(&Eh[(f * 216 + q) * 16 + 2 * c], pr, 2 * sizeof(LT));
        }
    }
    __syncthreads();
    const int g = lane >> 4;
    int qn[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        int x, y, z;
        morton_decode((uint32_t)(16 * nb + (lane & 15)), x, y, z);
        qn[nb] = ((x + 1) * 6 + (y + 1)) * 6 + (z + 1);
    }
    floatx4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const LT *Ehw = Eh + w * 216 * 16 + 8 * (g & 1);
#pragma unroll
    for (int ks = 0; ks < 13; ++ks) {   // source parents in the k order of the split-BF16 kernel
        const int q = 2 * ks + (g >> 1), d = q == 13 ? 26 : (q == 26 ? 13 : q);
        const int dq = ((d / 9 - 1) * 6 + ((d / 3) % 3 - 1)) * 6 + (d % 3 - 1);
        LT av[8];
        __builtin_memcpy(av, &a[ks], 16);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_lp32<LT>(av, Ehw + (qn[nb] + dq) * 16, acc[nb]);
    }
    const float u = unscale[f0 + w] * back;
    __syncthreads();
    float *Os = (float *)Eh;   // [parent][c_t][f][re/im]: 512 boxes x PF frequencies (16 KB)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int n = 16 * nb + (lane & 15);
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const int row = 4 * g + vv;
            Os[((n * 8 + (row >> 1)) * PF + w) * 2 + (row & 1)] = acc[nb][vv] * u;
        }
    }
    __syncthreads();
    for (int e = tid; e < 512 * 2; e += 256) {
        const int bl = e >> 1, half = e & 1;
        ((float4 *)(P + (512 * pt + bl) * nfp + f0))[half] = ((const float4 *)Os)[bl * 2 + half];
    }
}

// Transforms between the lattice values of a box (m0^3 equivalent densities or check
// potentials, C order (x, y, z), rows of m0^3 padded to 32 floats) and its spectrum on the
// cyclic N^3 grid, N = 2 m0 - 1.  The lattice values are real, so X(-k) = conj X(k): only
// the frequencies of one half are stored, and within the plane kz = 0 only one of each
// conjugate pair (H = m0 - 1):
//   kz = 1 .. H                      at f = (kx N + ky) H + kz - 1
//   kz = 0, kx = 0, ky = 0 .. H      at f = N^2 H + ky
//   kz = 0, kx = 1 .. H, any ky      at f = N^2 H + m0 + (kx - 1) N + ky
// (the other half of the plane kz = 0 is read back as the conjugate of its mirror
// (-kx, -ky)).  The pointwise products of real kernels and real densities have the same
// symmetry, so they too are computed at these frequencies only.  Separable, one wave per
// box (four per workgroup): each lane holds one line of a stage in registers and forms all
// its outputs, with the twiddles as immediates (every loop over cells and frequencies is
// unrolled); LDS carries the two hand-offs between stages.  The spectra rows hold the NF
// stored frequencies padded to nfp (a multiple of 16) complex values, the padding written
// as zeros.
template <int M>
struct LatticeDims {
    static constexpr int N = 2 * M - 1, H = M - 1, M3 = M * M * M;
    static constexpr int B0 = N * N * H;                       // first frequency of the plane kz = 0
    static constexpr int NF = B0 + M + H * N, NFP = (NF + 15) / 16 * 16;
    static constexpr int NM = N * M;                           // columns (ky, kz) of the x stage
    static constexpr int ROW = (M3 + 31) / 32 * 32;            // lattice row length
};

// Stored position of frequency (kx, ky, kz), and whether it is read as the conjugate of its
// mirror (kz = 0 only)
template <int M>
__device__ __forceinline__ int lattice_freq(int kx, int ky, int kz, bool &conj) {
    using L = LatticeDims<M>;
    constexpr int N = L::N, H = L::H;
    conj = false;
    if (kz > 0) return (kx * N + ky) * H + kz - 1;
    if (kx == 0) {
        conj = ky > H;
        return L::B0 + (conj ? N - ky : ky);
    }
    if (kx <= H) return L::B0 + M + (kx - 1) * N + ky;
    conj = true;
    return L::B0 + M + (N - kx - 1) * N + (N - ky) % N;
}

// cos and sin of 2 pi m / N, m < N, for the odd N = 2 m0 - 1 of m0 = 3 .. 8
template <int N>
struct TwTab;
template <>
struct TwTab<5> {
    static constexpr float c[5] = {1.000000000e+00f, 3.090169944e-01f, -8.090169944e-01f, -8.090169944e-01f, 3.090169944e-01f};
    static constexpr float s[5] = {0.000000000e+00f, 9.510565163e-01f, 5.877852523e-01f, -5.877852523e-01f, -9.510565163e-01f};
};
template <>
struct TwTab<7> {
    static constexpr float c[7] = {1.000000000e+00f, 6.234898019e-01f, -2.225209340e-01f, -9.009688679e-01f, -9.009688679e-01f, -2.225209340e-01f, 6.234898019e-01f};
    static constexpr float s[7] = {0.000000000e+00f, 7.818314825e-01f, 9.749279122e-01f, 4.338837391e-01f, -4.338837391e-01f, -9.749279122e-01f, -7.818314825e-01f};
};
template <>
struct TwTab<9> {
    static constexpr float c[9] = {1.000000000e+00f, 7.660444431e-01f, 1.736481777e-01f, -5.000000000e-01f, -9.396926208e-01f, -9.396926208e-01f, -5.000000000e-01f, 1.736481777e-01f, 7.660444431e-01f};
    static constexpr float s[9] = {0.000000000e+00f, 6.427876097e-01f, 9.848077530e-01f, 8.660254038e-01f, 3.420201433e-01f, -3.420201433e-01f, -8.660254038e-01f, -9.848077530e-01f, -6.427876097e-01f};
};
template <>
struct TwTab<11> {
    static constexpr float c[11] = {1.000000000e+00f, 8.412535328e-01f, 4.154150130e-01f, -1.423148383e-01f, -6.548607339e-01f, -9.594929736e-01f, -9.594929736e-01f, -6.548607339e-01f, -1.423148383e-01f, 4.154150130e-01f, 8.412535328e-01f};
    static constexpr float s[11] = {0.000000000e+00f, 5.406408175e-01f, 9.096319954e-01f, 9.898214419e-01f, 7.557495744e-01f, 2.817325568e-01f, -2.817325568e-01f, -7.557495744e-01f, -9.898214419e-01f, -9.096319954e-01f, -5.406408175e-01f};
};
template <>
struct TwTab<13> {
    static constexpr float c[13] = {1.000000000e+00f, 8.854560257e-01f, 5.680647467e-01f, 1.205366803e-01f, -3.546048870e-01f, -7.485107482e-01f, -9.709418174e-01f, -9.709418174e-01f, -7.485107482e-01f, -3.546048870e-01f, 1.205366803e-01f, 5.680647467e-01f, 8.854560257e-01f};
    static constexpr float s[13] = {0.000000000e+00f, 4.647231720e-01f, 8.229838659e-01f, 9.927088741e-01f, 9.350162427e-01f, 6.631226582e-01f, 2.393156643e-01f, -2.393156643e-01f, -6.631226582e-01f, -9.350162427e-01f, -9.927088741e-01f, -8.229838659e-01f, -4.647231720e-01f};
};
template <>
struct TwTab<15> {
    static constexpr float c[15] = {1.000000000e+00f, 9.135454576e-01f, 6.691306064e-01f, 3.090169944e-01f, -1.045284633e-01f, -5.000000000e-01f, -8.090169944e-01f, -9.781476007e-01f, -9.781476007e-01f, -8.090169944e-01f, -5.000000000e-01f, -1.045284633e-01f, 3.090169944e-01f, 6.691306064e-01f, 9.135454576e-01f};
    static constexpr float s[15] = {0.000000000e+00f, 4.067366431e-01f, 7.431448255e-01f, 9.510565163e-01f, 9.945218954e-01f, 8.660254038e-01f, 5.877852523e-01f, 2.079116908e-01f, -2.079116908e-01f, -5.877852523e-01f, -8.660254038e-01f, -9.945218954e-01f, -9.510565163e-01f, -7.431448255e-01f, -4.067366431e-01f};
};

// LDS hand-off between the lanes of one wave
__device__ __forceinline__ void lattice_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int LBW = 4;   // boxes per workgroup of the lattice transforms: one per wave

template <int M>
__global__ __launch_bounds__(256) void m2l_lattice_forward_kernel(const float *__restrict__ dens, int64_t nbx,
                                                                  const uint8_t *__restrict__ in_nz,
                                                                  float2 *__restrict__ E) {
    using L = LatticeDims<M>;
    using T = TwTab<L::N>;
    constexpr int N = L::N, NM = L::NM, MM = M * M;
    __shared__ float2 Z[LBW][L::M3];      // [kz][x][y]
    __shared__ float2 Y[LBW][M * NM];     // [x][ky][kz]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t box = (int64_t)blockIdx.x * LBW + w;
    if (box >= nbx || (in_nz && !in_nz[box])) return;   // never read: zero boxes are skipped
    if (lane < MM) {   // z: lane = (x, y), real in, kz = 0..M-1
        const float *src = dens + box * L::ROW + lane * M;
        float v[M];
#pragma unroll
        for (int z = 0; z < M; ++z) v[z] = src[z];
#pragma unroll
        for (int kz = 0; kz < M; ++kz) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int z = 0; z < M; ++z) {
                re = fmaf(v[z], T::c[(kz * z) % N], re);
                im = fmaf(-v[z], T::s[(kz * z) % N], im);
            }
            Z[w][kz * MM + lane] = make_float2(re, im);
        }
    }
    lattice_wave_sync();
    if (lane < MM) {   // y: lane = (x, kz), ky = 0..N-1
        const int x = lane / M, kz = lane % M;
        float2 v[M];
#pragma unroll
        for (int y = 0; y < M; ++y) v[y] = Z[w][kz * MM + x * M + y];
#pragma unroll
        for (int ky = 0; ky < N; ++ky) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int y = 0; y < M; ++y) {
                const float c = T::c[(ky * y) % N], sv = T::s[(ky * y) % N];
                re = fmaf(v[y].x, c, fmaf(v[y].y, sv, re));
                im = fmaf(v[y].y, c, fmaf(-v[y].x, sv, im));
            }
            Y[w][x * NM + ky * M + kz] = make_float2(re, im);
        }
    }
    lattice_wave_sync();
    float2 *dst = E + box * L::NFP;
    for (int c = lane; c < NM; c += 64) {   // x: lane = column (ky, kz), kx = 0..N-1
        const int ky = c / M, kz = c % M;
        float2 v[M];
#pragma unroll
        for (int x = 0; x < M; ++x) v[x] = Y[w][x * NM + c];
#pragma unroll
        for (int kx = 0; kx < N; ++kx) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int x = 0; x < M; ++x) {
                const float cv = T::c[(kx * x) % N], sv = T::s[(kx * x) % N];
                re = fmaf(v[x].x, cv, fmaf(v[x].y, sv, re));
                im = fmaf(v[x].y, cv, fmaf(-v[x].x, sv, im));
            }
            bool mirrored;
            const int f = lattice_freq<M>(kx, ky, kz, mirrored);
            if (!mirrored) dst[f] = make_float2(re, im);
        }
    }
    for (int f = L::NF + lane; f < L::NFP; f += 64) dst[f] = make_float2(0.f, 0.f);
}

// Inverse: the real lattice values (1 / N^3) sum_f w_kz Re(P(f) e^{+i theta}), w_kz = 1 at
// kz = 0 and 2 above (the conjugate half); the padding values of a row are zeros, and so is
// the whole row of a box that is not wanted.
template <int M>
__global__ __launch_bounds__(256) void m2l_lattice_inverse_kernel(const float2 *__restrict__ P, int64_t nbx,
                                                                  const uint8_t *__restrict__ out_need,
                                                                  float *__restrict__ dens) {
    using L = LatticeDims<M>;
    using T = TwTab<L::N>;
    constexpr int N = L::N, NM = L::NM, MM = M * M;
    __shared__ float2 A[LBW][M * NM];   // [x][ky][kz]
    __shared__ float2 B[LBW][L::M3];    // [x][y][kz]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t box = (int64_t)blockIdx.x * LBW + w;
    if (box >= nbx) return;
    float *dst = dens + box * L::ROW;
    if (out_need && !out_need[box]) {
        for (int j = lane; j < L::ROW; j += 64) dst[j] = 0.f;
        return;
    }
    const float2 *src = P + box * L::NFP;
    for (int c = lane; c < NM; c += 64) {   // x: lane = column (ky, kz), e^{+i theta}
        const int ky = c / M, kz = c % M;
        // stored positions of the column's frequencies (as lattice_freq, with kx a constant
        // of the unrolled loop: one select per frequency, every load unconditional)
        constexpr int H = L::H;
        const int lin = ky * H + kz - 1;                              // kz > 0: + kx N H
        const int p0 = L::B0 + (ky <= H ? ky : N - ky);               // kz = 0, kx = 0
        const int qb = L::B0 + M - N + ky;                            // kz = 0, kx <= H: + kx N
        const int rb = L::B0 + M + (N - 1) * N + (N - ky) % N;        // kz = 0, kx > H: - kx N
        float2 u[N];
#pragma unroll
        for (int kx = 0; kx < N; ++kx) {
            const int f0 = kx == 0 ? p0 : (kx <= H ? qb + kx * N : rb - kx * N);
            const bool cj = kz == 0 && (kx == 0 ? ky > H : kx > H);   // the conjugate of its mirror
            const float2 v = src[kz > 0 ? lin + kx * N * H : f0];
            u[kx] = make_float2(v.x, cj ? -v.y : v.y);
        }
#pragma unroll
        for (int x = 0; x < M; ++x) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int kx = 0; kx < N; ++kx) {
                const float cv = T::c[(kx * x) % N], sv = T::s[(kx * x) % N];
                re = fmaf(u[kx].x, cv, fmaf(-u[kx].y, sv, re));
                im = fmaf(u[kx].y, cv, fmaf(u[kx].x, sv, im));
            }
            A[w][x * NM + c] = make_float2(re, im);
        }
    }
    lattice_wave_sync();
    if (lane < MM) {   // y: lane = (x, kz)
        const int x = lane / M, kz = lane % M;
        float2 u[N];
#pragma unroll
        for (int ky = 0; ky < N; ++ky) u[ky] = A[w][x * NM + ky * M + kz];
#pragma unroll
        for (int y = 0; y < M; ++y) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int ky = 0; ky < N; ++ky) {
                const float cv = T::c[(ky * y) % N], sv = T::s[(ky * y) % N];
                re = fmaf(u[ky].x, cv, fmaf(-u[ky].y, sv, re));
                im = fmaf(u[ky].y, cv, fmaf(u[ky].x, sv, im));
            }
            B[w][(x * M + y) * M + kz] = make_float2(re, im);
        }
    }
    lattice_wave_sync();
    if (lane < MM) {   // z: lane = (x, y), the real part
        float2 u[M];
#pragma unroll
        for (int kz = 0; kz < M; ++kz) u[kz] = B[w][lane * M + kz];
        constexpr float inv = 1.0f / (float)(N * N * N);
#pragma unroll
        for (int z = 0; z < M; ++z) {
            float acc = 0.f;
#pragma unroll
            for (int kz = 0; kz < M; ++kz) {
                const float wgt = kz == 0 ? inv : 2.f * inv;
                acc = fmaf(u[kz].x, wgt * T::c[(kz * z) % N], fmaf(-u[kz].y, wgt * T::s[(kz * z) % N], acc));
            }
            dst[lane * M + z] = acc;
        }
    }
    for (int j = L::M3 + lane; j < L::ROW; j += 64) dst[j] = 0.f;
}

template <int M>
int launch_lattice(int dir, const float *in, int64_t nbx, int nfp, int row, const uint8_t *flags, float *out,
                   hipStream_t st) {
    using L = LatticeDims<M>;
    if (nfp != L::NFP || row != L::ROW)
        return fail(KIFMM_EINVAL, "lattice transform: spectrum or lattice row length does not match m0");
    const unsigned grid = (unsigned)((nbx + LBW - 1) / LBW);
    if (dir == 0)
        hipLaunchKernelGGL(m2l_lattice_forward_kernel<M>, dim3(grid), dim3(256), 0, st, in, nbx, flags, (float2 *)out);
    else
        hipLaunchKernelGGL(m2l_lattice_inverse_kernel<M>, dim3(grid), dim3(256), 0, st, (const float2 *)in, nbx, flags,
                           out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace

// dir 0: lattice values [nbx][row] -> spectra [nbx][nfp] complex at the stored frequencies
// (boxes with in_nz = 0 skipped); dir 1: spectra -> lattice values (boxes with out_need = 0
// written as zeros).  m0 in [3, 8], row = m0^3 padded to 32.
int run_m2l_lattice(int dir, int m0, const float *in, int64_t nbx, int nfp, int row, const uint8_t *flags,
                    float *out, hipStream_t st) {
    if (nbx <= 0) return KIFMM_OK;
    switch (m0) {
    case 3: return launch_lattice<3>(dir, in, nbx, nfp, row, flags, out, st);
    case 4: return launch_lattice<4>(dir, in, nbx, nfp, row, flags, out, st);
    case 5: return launch_lattice<5>(dir, in, nbx, nfp, row, flags, out, st);
    case 6: return launch_lattice<6>(dir, in, nbx, nfp, row, flags, out, st);
    case 7: return launch_lattice<7>(dir, in, nbx, nfp, row, flags, out, st);
    case 8: return launch_lattice<8>(dir, in, nbx, nfp, row, flags, out, st);
    default: return fail(KIFMM_EINVAL, "lattice transform: m0 must lie in [3, 8]");
    }
}

int run_m2l_pair_bf16x3(const float *E, const float *Ab, int nl, int nfp, const uint8_t *out_need,
                        const uint8_t *in_nz, float *P, hipStream_t st) {
    if (nl < 8 || (nl & (nl - 1)) != 0) return fail(KIFMM_EINVAL, "M2L spectra: boxes per axis must be 8, 16, ...");
    if (nfp % PF != 0) return fail(KIFMM_EINVAL, "M2L spectra: frequency count not a multiple of 4");
    if (!Ab) return fail(KIFMM_EINVAL, "M2L spectra: no split-BF16 operator fragments");
    const int64_t ntile = (int64_t)nl * nl * nl / 512;
    hipLaunchKernelGGL(m2l_pair_bf16x3_kernel, dim3((unsigned)ntile, (unsigned)(nfp / PF)), dim3(256), 0, st,
                       (const float2 *)E, (const uint16_t *)Ab, nl, nfp, out_need, in_nz, (float2 *)P);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_m2l_pair_lp1(int fp16, const float *E, const void *Al, const float *unscale, int nl, int nfp,
                     const uint8_t *out_need, const uint8_t *in_nz, float *P, hipStream_t st) {
    if (nl < 8 || (nl & (nl - 1)) != 0) return fail(KIFMM_EINVAL, "M2L spectra: boxes per axis must be 8, 16, ...");
    if (nfp % PF != 0) return fail(KIFMM_EINVAL, "M2L spectra: frequency count not a multiple of 4");
    if (!Al || !unscale) return fail(KIFMM_EINVAL, "M2L spectra: no single-part operator fragments");
    const int64_t ntile = (int64_t)nl * nl * nl / 512;
    const dim3 grid((unsigned)ntile, (unsigned)(nfp / PF));
    if (fp16)
        hipLaunchKernelGGL(m2l_pair_lp1_kernel<_Float16>, grid, dim3(256), 0, st, (const float2 *)E,
                           (const _Float16 *)Al, unscale, nl, nfp, out_need, in_nz, (float2 *)P);
    else
        hipLaunchKernelGGL(m2l_pair_lp1_kernel<__bf16>, grid, dim3(256), 0, st, (const float2 *)E, (const __bf16 *)Al,
                           unscale, nl, nfp, out_need, in_nz, (float2 *)P);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

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
