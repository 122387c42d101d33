// Near field in the Fourier domain (eq. (nearfar), direct part, with the self cell).
//
// On a uniform grid the near-range matrix between a target leaf and the leaf at offset o
// (in leaves) has entries G(cell_i - cell_j - 8 o) that depend on i - j only: it applies
// the kernel restricted to the differences d in [-7, 7]^3 + 8 o, a convolution.  On the
// cyclic grid of 15 points per axis (the fewest that keep the 15 differences per axis
// apart) those differences never wrap onto one another, so
//     S_t = inverse DFT( sum over the 27 neighbours o of Gh_o * DFT(q_{t+o}) )
// restricted to the 8^3 cells of t, with Gh_o the half spectrum (15 x 15 x 8 complex
// values) of the kernel of offset o, the self value included.  It is the same sum as the
// dense near field up to FP32 rounding, with about a fourteenth of its arithmetic per leaf
// (separable transforms and 27 complex products per frequency, against 27 dense 512 x 512
// products).
//
// Frequencies (kx, ky, kz), kz <= 7, are stored per leaf at f = (ky * 8 + kz) * 16 + kx:
// 120 columns (ky, kz) of 16 slots, the last slot of each zero.  The sources and the kernel
// are real, so X(-k) = conj X(k): the columns (ky, 0) with ky = 8 .. 14 are the conjugates of
// the columns (15 - ky, 0), slots reversed.  They are neither written by the forward
// transform nor multiplied (113 columns are), and the inverse transform reads them back as
// conjugates.
//
//   near_forward_kernel   one wave per source leaf: z, y and x transforms of the 8^3 values
//                         zero-padded to 15^3, each lane holding a line in registers and
//                         forming all its frequencies (twiddles as immediates); writes
//                         the 113 stored columns.
//   near_products_kernel  one workgroup per aligned 4^3 block of target leaves and the 16
//                         frequencies of one (ky, kz): the spectra of the 6^3 leaves around
//                         the block and 14 of the 27 kernel spectra are staged in LDS (the
//                         kernel is even and real, so the spectrum of offset -o is the
//                         conjugate of that of o: a column (ox, oy) and its mirror share
//                         their three kernel values); lane = 16 frequencies x 16 columns of
//                         4 targets along z (the 12 taps of a column at one (ox, oy) read 6
//                         source spectra).
//                         A workgroup takes 8 or 7 chunks of 16 frequencies (15 per
//                         block: 8 x 8 + 7 x 7 = 113 columns) in turn, the next
//                         chunk's spectra in flight (registers) while one is multiplied;
//                         XCD-contiguous order of the workgroups.
//                         Each chunk ends with the first inverse stage (over kx, at the 8
//                         cells x of the leaf), so 8 values per (ky, kz) are written.
//   near_inverse_kernel   one wave per target leaf: the y and z inverse transforms, only
//                         the 8^3 cells of the leaf.
#include "common.h"

namespace kifmm {

namespace {

// cos and sin of 2 pi m / 15, m = 0..14, for twiddles whose index differs between lanes
__constant__ float kCos15[15] = {1.000000000f, 0.913545458f, 0.669130606f, 0.309016994f, -0.104528463f, -0.500000000f, -0.809016994f, -0.978147601f, -0.978147601f, -0.809016994f, -0.500000000f, -0.104528463f, 0.309016994f, 0.669130606f, 0.913545458f};
__constant__ float kSin15[15] = {0.000000000f, 0.406736643f, 0.743144825f, 0.951056516f, 0.994521895f, 0.866025404f, 0.587785252f, 0.207911691f, -0.207911691f, -0.587785252f, -0.866025404f, -0.994521895f, -0.951056516f, -0.743144825f, -0.406736643f};

constexpr int NCOL = 120;       // columns (ky, kz): 15 x 8
constexpr int NF = NCOL * 16;   // frequency slots per leaf
constexpr int NKEEP = 113;      // stored columns: all but (ky, 0) for ky = 8 .. 14

// column of the j-th stored column: columns 0 .. 63 (ky < 8), then for ky = 8 .. 14 the
// columns kz = 1 .. 7
__device__ __forceinline__ int kept_column(int j) {
    if (j < 64) return j;
    const int t = j - 64;
    return 64 + 8 * (t / 7) + 1 + t % 7;
}

// The same values as compile-time constants: with every loop over frequencies and cells
// unrolled, each twiddle is an immediate operand.
constexpr float kC15[15] = {1.000000000e+00f, 9.135454576e-01f, 6.691306064e-01f, 3.090169944e-01f, -1.045284633e-01f, -5.000000000e-01f, -8.090169944e-01f, -9.781476007e-01f, -9.781476007e-01f, -8.090169944e-01f, -5.000000000e-01f, -1.045284633e-01f, 3.090169944e-01f, 6.691306064e-01f, 9.135454576e-01f};
constexpr float kS15[15] = {0.000000000e+00f, 4.067366431e-01f, 7.431448255e-01f, 9.510565163e-01f, 9.945218954e-01f, 8.660254038e-01f, 5.877852523e-01f, 2.079116908e-01f, -2.079116908e-01f, -5.877852523e-01f, -8.660254038e-01f, -9.945218954e-01f, -9.510565163e-01f, -7.431448255e-01f, -4.067366431e-01f};

// LDS handoff between the lanes of one wave (the transforms below use no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int LPW = 4;   // leaves per workgroup of the transforms: one per wave

// One wave per leaf.  z: lane = (x, y) reads its 8 contiguous values and forms kz = 0..7;
// y: lane = (x, kz) forms ky = 0..14 (twiddles as immediates); x: 15 groups of 8 columns
// (ky, kz), lane = (column, slot pair).  Each lane keeps its inputs in registers, so LDS
// carries only the hand-offs.
// GRID: the sources are read from the grid-order field I (n^3 cells, times vol) instead of
// the leaf-ordered q = vol I, the same FP32 values: the near field then needs no way in.
template <bool GRID>
__global__ __launch_bounds__(256) void near_forward_kernel(const float *__restrict__ q, const uint8_t *__restrict__ in_nz,
                                                           int64_t nleaf, float2 *__restrict__ Q, int n, float vol) {
    __shared__ float2 W[LPW][8 * NCOL];   // per wave: Z [kz][x][y], then Y [x][ky][kz]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t leaf = (int64_t)blockIdx.x * LPW + w;
    if constexpr (GRID) {   // the 4 waves take 4 leaves in a row along z: whole 128-byte lines of I
        const int nb = n >> 3, q4 = nb >> 2;
        const int64_t gq = blockIdx.x;
        const int lx = (int)(gq / ((int64_t)nb * q4)), ly = (int)((gq / q4) % nb), lz = 4 * (int)(gq % q4) + w;
        leaf = morton_encode(lx, ly, lz);
    }
    if (leaf >= nleaf || (in_nz && !in_nz[leaf])) return;   // never read: the products skip zero leaves
    float2 *Wb = W[w];
    {
        const float4 *src;
        if constexpr (GRID) {   // the leaf's line (x, y) = (lane / 8, lane % 8): 8 cells along z
            int lx, ly, lz;
            morton_decode((uint32_t)leaf, lx, ly, lz);
            src = (const float4 *)(q + ((int64_t)(8 * lx + (lane >> 3)) * n + 8 * ly + (lane & 7)) * n + 8 * lz);
        } else {
            src = (const float4 *)(q + leaf * 512 + lane * 8);
        }
        float4 a = src[0], b = src[1];
        if constexpr (GRID) {   // rounded products, as stored in q (never contracted into the sums)
#pragma clang fp contract(off)
            a = make_float4(a.x * vol, a.y * vol, a.z * vol, a.w * vol);
            b = make_float4(b.x * vol, b.y * vol, b.z * vol, b.w * vol);
        }
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int kz = 0; kz < 8; ++kz) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                re = fmaf(v[z], kC15[(kz * z) % 15], re);
                im = fmaf(-v[z], kS15[(kz * z) % 15], im);
            }
            Wb[kz * 64 + lane] = make_float2(re, im);
        }
    }
    wave_sync();
    {
        const int x = lane >> 3, kz = lane & 7;
        float2 v[8];
#pragma unroll
        for (int y = 0; y < 8; ++y) v[y] = Wb[kz * 64 + x * 8 + y];
        wave_sync();   // Y overwrites Z
        float2 s0 = make_float2(0.f, 0.f);   // ky = 0
#pragma unroll
        for (int y = 0; y < 8; ++y) s0 = make_float2(s0.x + v[y].x, s0.y + v[y].y);
        Wb[x * NCOL + kz] = s0;
        // ky and 15 - ky from the same four sums: with theta = 2 pi ky y / 15,
        // out(ky) = sum v e^{-i theta}, out(15 - ky) = sum v e^{+i theta}
#pragma unroll
        for (int ky = 1; ky < 8; ++ky) {
            float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                const float cv = kC15[(ky * y) % 15], sv = kS15[(ky * y) % 15];
                a = fmaf(v[y].x, cv, a);
                b = fmaf(v[y].y, sv, b);
                c = fmaf(v[y].y, cv, c);
                d = fmaf(v[y].x, sv, d);
            }
            Wb[x * NCOL + ky * 8 + kz] = make_float2(a + b, c - d);
            Wb[x * NCOL + (15 - ky) * 8 + kz] = make_float2(a - b, c + d);
        }
    }
    wave_sync();
    // x: lane = (column of a group of 8, kp): the slots kp and 15 - kp of the column from the
    // same four sums (kp = 0: kx = 0 and the zero slot 15); the wave's two stores cover 8
    // whole columns (1 KB)
    const int kp = lane & 7;
    float cw[8], sw[8];   // twiddles of kx = kp
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int m = (kp * x) % 15;
        cw[x] = kCos15[m];
        sw[x] = kSin15[m];
    }
    float2 *dst = Q + leaf * NF + kp;
#pragma unroll 3
    for (int g = 0; g < NCOL / 8; ++g) {
        const int r = 8 * g + (lane >> 3);   // column ky * 8 + kz
        float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            const float2 v = Wb[x * NCOL + r];
            a = fmaf(v.x, cw[x], a);
            b = fmaf(v.y, sw[x], b);
            c = fmaf(v.y, cw[x], c);
            d = fmaf(v.x, sw[x], d);
        }
        if (g < 8 || (lane >> 3) != 0) {   // (ky, 0) with ky >= 8: the mirror of (15 - ky, 0)
            dst[r * 16] = make_float2(a + b, c - d);
            dst[r * 16 + 15 - 2 * kp] = kp == 0 ? make_float2(0.f, 0.f) : make_float2(a - b, c + d);
        }
    }
}

constexpr int NCH = 8;    // frequency chunks per products workgroup (7 in the last 7 groups)
constexpr int NGRP = 15;  // workgroups per block of target leaves: 8 x 8 + 7 x 7 = 113 chunks

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 5) void near_products_kernel(const float2 *__restrict__ Q, const float2 *__restrict__ Gh,
                                                            int nb, const uint8_t *__restrict__ out_need,
                                                            const uint8_t *__restrict__ in_nz, float2 *__restrict__ P) {
    // Es: [region leaf][kx]; after the products of a chunk it holds their sums,
    // [target][kx] (padded rows of 17, 64 x 17)
    __shared__ float2 Es[216 * 16];
    __shared__ float2 Gs[14 * 16];    // [offset][kx], offsets 0 .. 13 (26 - t is the conjugate of t)
    const int tid = threadIdx.x, lane = tid & 63;
    // Workgroups go to the 8 XCDs in turn; each XCD takes one contiguous eighth of the
    // (frequency chunks, block) pairs, blocks fastest, so the neighbouring blocks that share
    // source spectra run out of the same L2.
    const int64_t nblk = (int64_t)nb * nb * nb / 64, total = nblk * NGRP;
    const int64_t wg = blockIdx.x;
    const int64_t lin = total % 8 == 0 ? (wg % 8) * (total / 8) + wg / 8 : wg;
    const int64_t blk = lin % nblk;
    // this workgroup's chunks of 16 frequencies: stored columns j0 .. j1 - 1 (groups 0 .. 7
    // take 8 columns, groups 8 .. 14 the 7 stored columns of ky = 8 .. 14).  The two kinds
    // alternate in the order of the workgroups, so every XCD gets the same share of each.
    const int k = (int)(lin / nblk), cg = (k & 1) ? 8 + (k >> 1) : k >> 1;
    const int j0 = cg < 8 ? NCH * cg : 64 + 7 * (cg - 8), j1 = cg < 8 ? j0 + NCH : j0 + 7;
    if (out_need) {   // the same ballot in every wave: all return or none
        if (__ballot(out_need[64 * blk + lane] != 0) == 0) return;
    }
    int bx, by, bz;
    morton_decode((uint32_t)blk, bx, by, bz);
    bx = 4 * bx - 1;
    by = 4 * by - 1;
    bz = 4 * bz - 1;
    // this thread's share of the staging: region leaves of e = tid + 256 i (8 float4 each);
    // leaves outside the grid and zero leaves are not read
    const float4 *src[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int e = tid + 256 * i, r = e >> 3;
        src[i] = nullptr;
        if (e < 216 * 8) {
            const int x = bx + r / 36, y = by + (r / 6) % 6, z = bz + r % 6;
            if (x >= 0 && y >= 0 && z >= 0 && x < nb && y < nb && z < nb) {
                const int64_t leaf = morton_encode(x, y, z);
                if (!in_nz || in_nz[leaf]) src[i] = (const float4 *)(Q + leaf * NF) + (e & 7);
            }
        }
    }
    const float4 *gsrc = tid < 14 * 8 ? (const float4 *)(Gh + (int64_t)(tid >> 3) * NF) + (tid & 7) : nullptr;
    float4 pre[7], gpre;
    auto fetch = [&](int c) {   // chunk c: frequencies 16 c .. 16 c + 15 (8 float4 per leaf)
#pragma unroll
        for (int i = 0; i < 7; ++i) pre[i] = src[i] ? src[i][c * 8] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (gsrc) gpre = gsrc[c * 8];
    };
    // the first inverse stage as an MFMA: this lane's entries of the real 32 x 16 DFT matrix
    // (k = 2 kx + re/im, n = 2 x + re/im; the padding slot kx = 15 has zero rows), in the
    // A-operand layout of v_mfma_f32_16x16x4f32 for the transposed product (row n = lane
    // % 16, k = 4 ks + lane / 16)
    const int g4 = lane >> 4, n16 = lane & 15;
    float wdft[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const int k = 4 * ks + g4, kx = k >> 1, x = n16 >> 1;
        const int m = (kx * x) % 15;
        const float cv = kCos15[m], sv = kSin15[m];
        const float re_row = (k & 1) ? -sv : cv, im_row = (k & 1) ? cv : sv;   // U += P e^{+i theta}
        wdft[ks] = kx >= 15 ? 0.f : ((n16 & 1) ? im_row : re_row);
    }
    // lane: frequency f and a column of 4 targets (a, b, 0..3) of the block, so that for
    // each (ox, oy) the 4 targets' 12 taps read 6 source spectra
    const int f = tid & 15, grp = tid >> 4, ta = grp >> 2, tb = grp & 3;
    int tl[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) tl[s] = (int)morton_encode(ta, tb, s);
    const int col = (((ta + 1) * 6 + (tb + 1)) * 6) * 16 + f;   // region (ta+1, tb+1, 0)
    fetch(kept_column(j0));
    for (int j = j0; j < j1; ++j) {
        const int c = kept_column(j);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            if (tid + 256 * i < 216 * 8) ((float4 *)Es)[tid + 256 * i] = pre[i];
        if (gsrc) ((float4 *)Gs)[tid] = gpre;
        __syncthreads();
        if (j + 1 < j1) fetch(kept_column(j + 1));   // in flight while this chunk is multiplied
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
        // (ox, oy) = column c of 9 and its mirror 8 - c: the kernel is even and real, so the
        // spectrum of offset -o is the conjugate of that of o (offset index 26 - t for t);
        // oz and the 4 targets share 6 sources per column
        auto column = [&](int oxy, const float2 (&g)[3], float sgn) {   // sgn -1: conjugates
            const int base = col + ((oxy / 3 - 1) * 36 + (oxy % 3 - 1) * 6) * 16;
            float2 e[6];
#pragma unroll
            for (int z = 0; z < 6; ++z) e[z] = Es[base + z * 16];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int oz = 0; oz < 3; ++oz) {   // source z = s + oz - 1, region z = s + oz
                    const float2 v = e[s + oz];
                    const float gy = sgn * g[oz].y;
                    ar[s] = fmaf(g[oz].x, v.x, fmaf(-gy, v.y, ar[s]));
                    ai[s] = fmaf(g[oz].x, v.y, fmaf(gy, v.x, ai[s]));
                }
        };
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float2 g[3], gm[3];
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) g[oz] = Gs[(c * 3 + oz) * 16 + f];
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) gm[oz] = g[2 - oz];
            column(c, g, 1.f);
            column(8 - c, gm, -1.f);
        }
        {   // the centre column: oz = +1 is the conjugate of oz = -1, oz = 0 the self offset
            float2 g[3];
            g[0] = Gs[12 * 16 + f];
            g[1] = Gs[13 * 16 + f];
            g[2] = make_float2(g[0].x, -g[0].y);
            column(4, g, 1.f);
        }
        __syncthreads();   // every wave is done with Es before Ps overwrites it
#pragma unroll
        for (int s = 0; s < 4; ++s) Es[tl[s] * 17 + f] = make_float2(ar[s], ai[s]);
        __syncthreads();
        // first inverse stage, over kx, at the 8 cells x of each target: this chunk holds all
        // 15 kx of one (ky, kz) = c, so U[leaf][c][x] = sum_kx P e^{+2 pi i kx x / 15}.  Wave
        // w: the 16 targets 16 w .. 16 w + 15, as U^T = W^T P^T over the reals (K = 32); the
        // B operand (k = 4 ks + lane / 16, target lane % 16) is read from Ps, and the lane's
        // 4 results (n = 4 (lane / 16) + v) are x = 2 (lane / 16), + 1, re and im.
        {
            const int w = tid >> 6, t = 16 * w + n16;
            const float *pt = (const float *)(Es + t * 17);
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wdft[ks], pt[(2 * ks + (g4 >> 1)) * 2 + (g4 & 1)], acc, 0, 0, 0);
            *(float4 *)(P + ((64 * blk + t) * NCOL + c) * 8 + 2 * g4) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
        __syncthreads();   // the staging of the next chunk overwrites Es, Gs and Ps
    }
}

// One wave per leaf.  y: lane = (kz, x) reads its 15 values (ky = 0..14) of the sums after
// the x stage, coalesced, and forms y = 0..7; z: lane = (x, y) forms the 8 real values
// along z (the conjugate half counted twice) and writes them, contiguous.
__global__ __launch_bounds__(256) void near_inverse_kernel(const float2 *__restrict__ U,
                                                           const uint8_t *__restrict__ out_need, int64_t nleaf,
                                                           float *__restrict__ S) {
    __shared__ float2 V[LPW][512];   // per wave: [x][y][kz]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t leaf = (int64_t)blockIdx.x * LPW + w;
    if (leaf >= nleaf || (out_need && !out_need[leaf])) return;   // never read: the final sum writes 0 there
    float2 *Vb = V[w];
    {
        const int kz = lane >> 3, x = lane & 7;
        float2 u[15];
#pragma unroll
        for (int ky = 0; ky < 15; ++ky) {   // [ky * 8 + kz][x]; (ky >= 8, 0): conj of (15 - ky, 0)
            const bool mirrored = ky >= 8 && kz == 0;
            u[ky] = U[leaf * NCOL * 8 + (mirrored ? 15 - ky : ky) * 64 + lane];
            if (mirrored) u[ky].y = -u[ky].y;
        }
        // ky and 15 - ky together: u(ky) e^{+i theta} + u(15 - ky) e^{-i theta}
        //   = (u(ky) + u(15 - ky)) cos theta + i (u(ky) - u(15 - ky)) sin theta
        float2 pk[8], mk[8];
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            pk[k] = make_float2(u[k].x + u[15 - k].x, u[k].y + u[15 - k].y);
            mk[k] = make_float2(u[k].x - u[15 - k].x, u[k].y - u[15 - k].y);
        }
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            float re = u[0].x, im = u[0].y;
#pragma unroll
            for (int k = 1; k < 8; ++k) {
                const float c = kC15[(k * y) % 15], sv = kS15[(k * y) % 15];
                re = fmaf(pk[k].x, c, fmaf(-mk[k].y, sv, re));
                im = fmaf(pk[k].y, c, fmaf(mk[k].x, sv, im));
            }
            Vb[(x * 8 + y) * 8 + kz] = make_float2(re, im);
        }
    }
    wave_sync();
    float2 v[8];
#pragma unroll
    for (int kz = 0; kz < 8; ++kz) v[kz] = Vb[lane * 8 + kz];
    float o[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        float acc = 0.f;
#pragma unroll
        for (int kz = 0; kz < 8; ++kz) {
            const float wgt = (kz == 0 ? 1.0f : 2.0f) / 3375.0f;
            acc = fmaf(v[kz].x, wgt * kC15[(kz * z) % 15], fmaf(-v[kz].y, wgt * kS15[(kz * z) % 15], acc));
        }
        o[z] = acc;
    }
    float4 *dst = (float4 *)(S + leaf * 512 + lane * 8);
    dst[0] = make_float4(o[0], o[1], o[2], o[3]);
    dst[1] = make_float4(o[4], o[5], o[6], o[7]);
}

}  // namespace

// stage 0: spectra of the sources, 1: products, 2: inverse transforms into S
int run_near_fft_stage(int stage, const float *q, const float *Gh, int nb, const uint8_t *out_need,
                       const uint8_t *in_nz, float *Qbuf, float *Pbuf, float *S, hipStream_t st, const float *I_grid,
                       float vol) {
    if (nb < 4 || (nb & (nb - 1)) != 0) return fail(KIFMM_EINVAL, "near-field spectra: leaves per axis must be 4, 8, 16, ...");
    const int64_t nleaf = (int64_t)nb * nb * nb;
    if (stage == 0 && I_grid)
        hipLaunchKernelGGL(near_forward_kernel<true>, dim3((unsigned)((nleaf + LPW - 1) / LPW)), dim3(256), 0, st,
                           I_grid, in_nz, nleaf, (float2 *)Qbuf, 8 * nb, vol);
    else if (stage == 0)
        hipLaunchKernelGGL(near_forward_kernel<false>, dim3((unsigned)((nleaf + LPW - 1) / LPW)), dim3(256), 0, st, q,
                           in_nz, nleaf, (float2 *)Qbuf, 0, 1.f);
    else if (stage == 1)
        hipLaunchKernelGGL(near_products_kernel, dim3((unsigned)(nleaf / 64 * NGRP)), dim3(256), 0, st,
                           (const float2 *)Qbuf, (const float2 *)Gh, nb, out_need, in_nz, (float2 *)Pbuf);
    else
        hipLaunchKernelGGL(near_inverse_kernel, dim3((unsigned)((nleaf + LPW - 1) / LPW)), dim3(256), 0, st,
                           (const float2 *)Pbuf, out_need, nleaf,
                           S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
