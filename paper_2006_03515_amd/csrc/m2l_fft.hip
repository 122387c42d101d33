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
// GEMMs; this file holds the pointwise part, which has no dense contraction to put on
// MFMA (each frequency is its own 189-tap stencil over the boxes).
//
//   m2l_hadamard_kernel  one workgroup per aligned 4^3 block of target boxes (64
//                        consecutive Morton indices) and FC frequencies.  The block's
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
        ar0 += kv.x * e0.x - kv.y * e0.y;
        ai0 += kv.x * e0.y + kv.y * e0.x;
        ar1 += kv.x * e1.x - kv.y * e1.y;
        ai1 += kv.x * e1.y + kv.y * e1.x;
    }
    P[(64 * blk + tl[0]) * nfp + f0 + f] = make_float2(ar0, ai0);
    P[(64 * blk + tl[1]) * nfp + f0 + f] = make_float2(ar1, ai1);
}

}  // namespace

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
