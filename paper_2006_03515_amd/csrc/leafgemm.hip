// The two leaf-level translations fused with the permutes between grid order and
// leaf order (FP32, leaves of 8^3 cells):
//
//   P2M (eq. (s2m) at the leaves) with the way in:
//       q[leaf][cell] = h^3 I[grid cell]            (written: the near field reads it)
//       c_u[leaf]     = A_p2m q[leaf]               A_p2m = U_u^T G(x^u, leaf cells), KU x 512
//   L2P (algorithm outline step 4, far part) with the sum and the way out:
//       S[grid cell]  = c (A_l2p c_d[leaf] + S_near[leaf][cell])   A_l2p = G(cells, y^d) V_d S^-1, 512 x KD
//
// Over all leaves each is one GEMM with a shared operator (K = 512 or KD), so a
// workgroup takes 32 Morton-consecutive leaves (an aligned block of 2 x 4 x 4 leaves
// along x, y, z) as the 32 columns of v_mfma_f32_32x32x2f32 tiles: the sources or the
// coefficients of the block are staged once in LDS, and each wave streams the operator
// rows of its 32-row tiles from L2 in MFMA fragment order (one contiguous 1 KB read per
// wave and 8-wide reduction chunk; the fragments are packed once at precompute).  The
// values cross HBM once: I in and q, c_u out for the way in; c_d, S_near in and S out
// for the way out.
//
// Fragment order of an operator A (rows x cols, row-major) for tile t (rows 32t ..
// 32t + 31) and chunk c (columns 8c .. 8c + 7): lane l = 32 h + r holds the float4
// A[32t + r][8c + 4h .. 8c + 4h + 3].  Its j-th component is the A operand of the j-th
// of four MFMA steps, whose B operand is component j of the float4 B[8c + 4h ..][col],
// so the four steps sum the chunk's 8 products (in a permuted order of the reduction
// index, the same for A and B).
//
// Split BF16 (precision KIFMM_BF16X3): each operand is the sum of two BF16 numbers, the
// value rounded to BF16 and the BF16 of what remains, and a product is A_hi B_hi + A_hi B_lo
// + A_lo B_hi on v_mfma_f32_32x32x16_bf16 with FP32 accumulation (about 16 mantissa bits
// per operand; the dropped A_lo B_lo is below 2^-16 of the product).  Fragments of tile t
// and 16-wide chunk c: lane l = 32 h + r holds in part 0 the BF16 high parts of
// A[32t + r][16c + 8h .. 16c + 8h + 7] and in part 1 their remainders, split from the FP64
// operator; the B operand of the lane is the same 8 reduction indices of its column, split
// while the block is staged in LDS.  The accumulator layout is that of the FP32 kernels.
#include "common.h"

namespace kifmm {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kLeafBlock = 32;    // leaves per workgroup
constexpr int kQRow = 129;        // LDS row of a leaf's sources: 128 float4 + 1 pad

__device__ inline float4 scaled(float4 v, float s) { return make_float4(v.x * s, v.y * s, v.z * s, v.w * s); }

// Morton offset (0..31) inside the block of leaf (dx, dy, dz), dx < 2, dy < 4, dz < 4: the
// block's codes differ in their five lowest bits, z0 y0 x0 z1 y1 from the least significant
__device__ inline int block_code(int dx, int dy, int dz) {
    return (dz & 1) | ((dy & 1) << 1) | (dx << 2) | ((dz >> 1) << 3) | ((dy >> 1) << 4);
}
__device__ inline void block_leaf(int m, int &dx, int &dy, int &dz) {
    dz = (m & 1) | (((m >> 3) & 1) << 1);
    dy = ((m >> 1) & 1) | (((m >> 4) & 1) << 1);
    dx = (m >> 2) & 1;
}

// 8-wide reduction chunks of the L2P operator: KD / 8 rounded up to even
__host__ __device__ inline int l2p_chunks(int KD) { return (KD / 8 + 1) & ~1; }

__device__ inline floatx16 mfma4(const float4 &a, const float4 &b, floatx16 acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
    return acc;
}

// fragments[(t * nchunk + c) * 64 + l] = A[32t + l % 32][8c + 4(l / 32) .. + 3]; rows and
// columns past the operator's size are zero
__global__ void pack_fragments_kernel(const float *__restrict__ A, int rows, int cols, int lda, int ntile,
                                      int nchunk, float4 *__restrict__ frag) {
    const int64_t total = (int64_t)ntile * nchunk * 64;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e & 63);
        const int64_t tc = e >> 6;
        const int c = (int)(tc % nchunk), t = (int)(tc / nchunk);
        const int r = 32 * t + (l & 31), k0 = 8 * c + 4 * (l >> 5);
        float v[4];
        for (int j = 0; j < 4; ++j) v[j] = (r < rows && k0 + j < cols) ? A[(int64_t)r * lda + k0 + j] : 0.f;
        frag[e] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// Way in + P2M.  Grid: one workgroup per block of 32 leaves (nleaf / 32 workgroups).
// n % 32 == 0, ntile = KU / 32 row tiles of A (fragments of 64 chunks of 8 columns).
__global__ __launch_bounds__(256, 2) void p2m_permute_in_kernel(const float *__restrict__ I, int n, float vol,
                                                                const float4 *__restrict__ Af, int ntile, int KU,
                                                                float *__restrict__ q, float *__restrict__ cu) {
    __shared__ float4 Qs[kLeafBlock * kQRow];
    const uint32_t g = blockIdx.x;
    int bx, by, bz;
    morton_decode(g << 5, bx, by, bz);
    const int tid = threadIdx.x;
    // the block's cells: 16 x 32 grid rows (i, j) of 32 cells along k (4 leaves' lines);
    // one thread reads a row's 128 contiguous bytes
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int r = tid + 256 * rr;
        const int ii = r >> 5, jj = r & 31;
        const float4 *src = (const float4 *)(I + ((int64_t)((bx << 3) + ii) * n + (by << 3) + jj) * n + (bz << 3));
        const int local = ((ii & 7) * 8 + (jj & 7)) * 8;   // first cell of the line in its leaf
        float4 v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = scaled(src[c], vol);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = block_code(ii >> 3, jj >> 3, c);
            if (q) {   // the leaf-ordered sources, when a later pass reads them
                float4 *dq = (float4 *)(q + ((int64_t)((g << 5) + m) << 9) + local);
                dq[0] = v[2 * c];
                dq[1] = v[2 * c + 1];
            }
            Qs[m * kQRow + (local >> 2)] = v[2 * c];
            Qs[m * kQRow + (local >> 2) + 1] = v[2 * c + 1];
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, col = lane & 31, h = lane >> 5;
    const float4 *bq = Qs + col * kQRow + h;
    for (int t = wave; t < ntile; t += 4) {
        const float4 *af = Af + (int64_t)t * 64 * 64 + lane;
        floatx16 acc;
        double tot[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) { acc[v] = 0.f; tot[v] = 0.0; }
        // 64 chunks in 8 groups of 8; the next group's operator fragments are loaded while
        // one group is multiplied.  FP32 MFMA partials are folded into FP64 every 16 chunks
        // (128 products per FP32 chain).
        float4 a[8], an[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = af[c * 64];
#pragma unroll 1
        for (int grp = 0; grp < 8; ++grp) {
            if (grp < 7) {
#pragma unroll
                for (int c = 0; c < 8; ++c) an[c] = af[((grp + 1) * 8 + c) * 64];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) acc = mfma4(a[c], bq[2 * (grp * 8 + c)], acc);
            if (grp & 1) {
#pragma unroll
                for (int v = 0; v < 16; ++v) { tot[v] += (double)acc[v]; acc[v] = 0.f; }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) a[c] = an[c];
        }
        // D layout of 32x32x2: lane holds column lane % 32 and, in registers 4g .. 4g + 3,
        // rows 8g + 4 (lane / 32) + 0..3
        float *o = cu + (int64_t)((g << 5) + col) * KU + 32 * t + 4 * h;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg)
            *(float4 *)(o + 8 * gg) = make_float4((float)tot[4 * gg], (float)tot[4 * gg + 1], (float)tot[4 * gg + 2],
                                                  (float)tot[4 * gg + 3]);
    }
}

// L2P + sum with the near field + way out.  Grid: one workgroup per block of 32 leaves.
// KD % 8 == 0, KD <= 256; the operator has 512 rows (16 tiles) and an even number of
// 8-wide chunks (KD rounded up to 16, the padding zero in the fragments and in the staged
// coefficients); wave w takes the cells 128 w .. 128 w + 127 of every leaf of the block
// (tiles 4w .. 4w + 3).
__global__ __launch_bounds__(256, 2) void l2p_permute_out_kernel(const float *__restrict__ cd, int KD,
                                                                 const float4 *__restrict__ Lf,
                                                                 const float *__restrict__ Snear, int n, float scale,
                                                                 const uint8_t *__restrict__ want, float *__restrict__ S) {
    __shared__ float4 Cs[kLeafBlock * 65];
    const int nchunk = l2p_chunks(KD), crow = 2 * nchunk + 1;
    const uint32_t g = blockIdx.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < kLeafBlock * 2 * nchunk; e += 256) {
        const int m = e / (2 * nchunk), k4 = e % (2 * nchunk);
        Cs[m * crow + k4] = 4 * k4 < KD ? ((const float4 *)(cd + (int64_t)((g << 5) + m) * KD))[k4]
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, col = lane & 31, h = lane >> 5;
    const float4 *bc = Cs + col * crow + h;
    // column col of the tiles is leaf 32 g + col
    const int leaf = (int)(g << 5) + col;
    int bx, by, bz, dx, dy, dz;
    morton_decode(g << 5, bx, by, bz);
    block_leaf(col, dx, dy, dz);
    const bool keep = !want || want[leaf];
    const float *sn = Snear + ((int64_t)leaf << 9);
    float *base = S + ((int64_t)((bx + dx) << 3) * n + ((by + dy) << 3)) * n + ((bz + dz) << 3);
    // The wave's operator fragments as one sequence of steps s = pr * nchunk + c (tiles
    // 4 wave + 2 pr + i, chunk c), requested two steps ahead into two register sets: the last
    // steps of the first pair request the second pair's first chunks, before the first pair's
    // sums are stored.  Loads complete in the order they were issued, so a step waits only
    // for its own fragments and what was issued before them, never for the stores or the
    // near-field loads that follow; the step index is clamped, so every load is issued
    // unconditionally (the clamped ones are repeats, never used).
    const float4 *lf = Lf + (int64_t)(4 * wave) * nchunk * 64 + lane;
    const int last = 2 * nchunk - 1;
    auto frag = [&](int st, int i) {
        st = min(st, last);
        const int pr = st >= nchunk ? 1 : 0;
        return lf[((int64_t)(2 * pr + i) * nchunk + st - pr * nchunk) * 64];
    };
    float4 a0[2], a1[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a0[i] = frag(0, i);
#pragma unroll
    for (int i = 0; i < 2; ++i) a1[i] = frag(1, i);
#pragma unroll 1
    for (int pr = 0; pr < 2; ++pr) {
        float4 sv[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int c = 128 * wave + 32 * (2 * pr + i) + 8 * gg + 4 * h;
                sv[i][gg] = *(const float4 *)(sn + c);   // every leaf's row exists; unwanted ones are not used
            }
        floatx16 ac[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) ac[i][v] = 0.f;
        for (int c = 0; c < nchunk; c += 2) {   // nchunk is even: chunk c in a0, c + 1 in a1
            const int st = pr * nchunk + c;
            const float4 b0 = bc[2 * c];
#pragma unroll
            for (int i = 0; i < 2; ++i) ac[i] = mfma4(a0[i], b0, ac[i]);
#pragma unroll
            for (int i = 0; i < 2; ++i) a0[i] = frag(st + 2, i);
            const float4 b1 = bc[2 * c + 2];
#pragma unroll
            for (int i = 0; i < 2; ++i) ac[i] = mfma4(a1[i], b1, ac[i]);
#pragma unroll
            for (int i = 0; i < 2; ++i) a1[i] = frag(st + 3, i);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int c = 128 * wave + 32 * (2 * pr + i) + 8 * gg + 4 * h;
                // a select, not a branch: unwanted leaves are written as zeros whatever their
                // (unwritten) near-field rows hold
                const float4 v = make_float4(keep ? (ac[i][4 * gg] + sv[i][gg].x) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 1] + sv[i][gg].y) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 2] + sv[i][gg].z) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 3] + sv[i][gg].w) * scale : 0.f);
                *(float4 *)(base + ((int64_t)(c >> 6) * n + ((c >> 3) & 7)) * n + (c & 7)) = v;
            }
    }
}

// 16-wide reduction chunks of the split-BF16 L2P operator: KD / 16 rounded up, then to even
__host__ __device__ inline int l2p_chunks_x3(int KD) { return ((KD + 15) / 16 + 1) & ~1; }

// FP32 -> BF16 bits, round to nearest even (finite values)
__device__ inline uint32_t bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// split-BF16 fragments: xf[((t * nck + c) * 2 + part) * 64 + l] holds part 0 (the BF16 of
// A[32t + l % 32][16c + 8(l / 32) + j], j = 0..7, two to a word) or part 1 (the BF16 of
// each value minus its part 0, formed in FP64); rows and columns past the operator's size
// are zero
__global__ void pack_fragments_x3_kernel(const double *__restrict__ A, int rows, int cols, int lda, int ntile,
                                         int nck, uint4 *__restrict__ xf) {
    const int64_t total = (int64_t)ntile * nck * 64;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e & 63);
        const int64_t tc = e >> 6;
        const int c = (int)(tc % nck), t = (int)(tc / nck);
        const int r = 32 * t + (l & 31), k0 = 16 * c + 8 * (l >> 5);
        uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
        for (int j = 0; j < 8; ++j) {
            const double a = (r < rows && k0 + j < cols) ? A[(int64_t)r * lda + k0 + j] : 0.0;
            const uint32_t hb = bf16_bits((float)a);
            const uint32_t lb = bf16_bits((float)(a - (double)__uint_as_float(hb << 16)));
            hw[j >> 1] |= hb << (16 * (j & 1));
            lw[j >> 1] |= lb << (16 * (j & 1));
        }
        xf[(tc * 2) * 64 + l] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        xf[(tc * 2 + 1) * 64 + l] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
}

// four FP32 values -> their BF16 high parts and remainders, two to a word
__device__ inline void split4(const float4 &v, uint2 &hi, uint2 &lo) {
    uint16_t h0, h1, h2, h3, l0, l1, l2, l3;
    split_bf16(v.x, h0, l0);
    split_bf16(v.y, h1, l1);
    split_bf16(v.z, h2, l2);
    split_bf16(v.w, h3, l3);
    hi = make_uint2((uint32_t)h0 | ((uint32_t)h1 << 16), (uint32_t)h2 | ((uint32_t)h3 << 16));
    lo = make_uint2((uint32_t)l0 | ((uint32_t)l1 << 16), (uint32_t)l2 | ((uint32_t)l3 << 16));
}

__device__ inline floatx16 mfma_x3(const uint4 &ah, const uint4 &al, const uint4 &bh, const uint4 &bl, floatx16 acc) {
    bf16x8 a_hi, a_lo, b_hi, b_lo;
    __builtin_memcpy(&a_hi, &ah, 16);
    __builtin_memcpy(&a_lo, &al, 16);
    __builtin_memcpy(&b_hi, &bh, 16);
    __builtin_memcpy(&b_lo, &bl, 16);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi, b_hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi, b_lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo, b_hi, acc, 0, 0, 0);
    return acc;
}

constexpr int kXRow = 65;   // LDS row of a leaf's split sources: 64 x 8 BF16 + 1 pad (16-byte units)

// Way in + P2M in split BF16: the same blocks, staging and outputs as p2m_permute_in_kernel;
// the sources are staged as BF16 high parts and remainders (two planes), and each wave's
// tiles take 32 chunks of 16 cells, the operator fragments two chunks ahead.  FP32
// partial sums are folded into FP64 every 8 chunks.
__global__ __launch_bounds__(256, 2) void p2m_permute_in_x3_kernel(const float *__restrict__ I, int n, float vol,
                                                                   const uint4 *__restrict__ Ax, int ntile, int KU,
                                                                   float *__restrict__ q, float *__restrict__ cu) {
    __shared__ uint4 Qh[kLeafBlock * kXRow], Ql[kLeafBlock * kXRow];
    const uint32_t g = blockIdx.x;
    int bx, by, bz;
    morton_decode(g << 5, bx, by, bz);
    const int tid = threadIdx.x;
    uint2 *qh2 = (uint2 *)Qh, *ql2 = (uint2 *)Ql;   // 8-byte units: 4 BF16 values
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int r = tid + 256 * rr;
        const int ii = r >> 5, jj = r & 31;
        const float4 *src = (const float4 *)(I + ((int64_t)((bx << 3) + ii) * n + (by << 3) + jj) * n + (bz << 3));
        const int local = ((ii & 7) * 8 + (jj & 7)) * 8;   // first cell of the line in its leaf
        float4 v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = scaled(src[c], vol);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = block_code(ii >> 3, jj >> 3, c);
            if (q) {
                float4 *dq = (float4 *)(q + ((int64_t)((g << 5) + m) << 9) + local);
                dq[0] = v[2 * c];
                dq[1] = v[2 * c + 1];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                uint2 hi, lo;
                split4(v[2 * c + u], hi, lo);
                qh2[m * 2 * kXRow + (local >> 2) + u] = hi;
                ql2[m * 2 * kXRow + (local >> 2) + u] = lo;
            }
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, col = lane & 31, h = lane >> 5;
    const uint4 *bh = Qh + col * kXRow + h, *bl = Ql + col * kXRow + h;   // chunk c: unit 2c + h
    for (int t = wave; t < ntile; t += 4) {
        const uint4 *af = Ax + (int64_t)t * 32 * 128 + lane;   // chunk c: part p at (2c + p) * 64
        floatx16 acc;
        double tot[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) { acc[v] = 0.f; tot[v] = 0.0; }
        uint4 a0h = af[0], a0l = af[64], a1h = af[128], a1l = af[192];
#pragma unroll 1
        for (int c = 0; c < 32; c += 2) {   // chunk c in set 0, c + 1 in set 1
            const int n0 = min(c + 2, 31), n1 = min(c + 3, 31);   // clamped: every load is issued
            acc = mfma_x3(a0h, a0l, bh[2 * c], bl[2 * c], acc);
            a0h = af[n0 * 128];
            a0l = af[n0 * 128 + 64];
            acc = mfma_x3(a1h, a1l, bh[2 * c + 2], bl[2 * c + 2], acc);
            a1h = af[n1 * 128];
            a1l = af[n1 * 128 + 64];
            if ((c & 7) == 6) {
#pragma unroll
                for (int v = 0; v < 16; ++v) { tot[v] += (double)acc[v]; acc[v] = 0.f; }
            }
        }
        float *o = cu + (int64_t)((g << 5) + col) * KU + 32 * t + 4 * h;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg)
            *(float4 *)(o + 8 * gg) = make_float4((float)tot[4 * gg], (float)tot[4 * gg + 1], (float)tot[4 * gg + 2],
                                                  (float)tot[4 * gg + 3]);
    }
}

// L2P + sum with the near field + way out in split BF16: the same blocks, wave tiles and
// epilogue as l2p_permute_out_kernel; the block's coefficients are staged as BF16 high
// parts and remainders (rows of 2 nck + 1 16-byte units), the chunks are 16 wide.
__global__ __launch_bounds__(256, 2) void l2p_permute_out_x3_kernel(const float *__restrict__ cd, int KD,
                                                                    const uint4 *__restrict__ Lx,
                                                                    const float *__restrict__ Snear, int n, float scale,
                                                                    const uint8_t *__restrict__ want,
                                                                    float *__restrict__ S) {
    __shared__ uint4 Ch[kLeafBlock * 33], Cl[kLeafBlock * 33];
    const int nck = l2p_chunks_x3(KD), crow = 2 * nck + 1;
    const uint32_t g = blockIdx.x;
    const int tid = threadIdx.x;
    uint2 *ch2 = (uint2 *)Ch, *cl2 = (uint2 *)Cl;
    for (int e = tid; e < kLeafBlock * 4 * nck; e += 256) {   // 4 nck float4 per leaf
        const int m = e / (4 * nck), k4 = e % (4 * nck);
        const float4 v = 4 * k4 < KD ? ((const float4 *)(cd + (int64_t)((g << 5) + m) * KD))[k4]
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
        uint2 hi, lo;
        split4(v, hi, lo);
        ch2[m * 2 * crow + k4] = hi;
        cl2[m * 2 * crow + k4] = lo;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, col = lane & 31, h = lane >> 5;
    const uint4 *bh = Ch + col * crow + h, *bl = Cl + col * crow + h;   // chunk c: unit 2c + h
    const int leaf = (int)(g << 5) + col;
    int bx, by, bz, dx, dy, dz;
    morton_decode(g << 5, bx, by, bz);
    block_leaf(col, dx, dy, dz);
    const bool keep = !want || want[leaf];
    const float *sn = Snear + ((int64_t)leaf << 9);
    float *base = S + ((int64_t)((bx + dx) << 3) * n + ((by + dy) << 3)) * n + ((bz + dz) << 3);
    // the wave's fragments as one sequence of steps st = pr * nck + c (tiles 4 wave + 2 pr +
    // i, chunk c), two steps ahead in two register sets, every load issued (clamped index)
    const uint4 *lf = Lx + (int64_t)(4 * wave) * nck * 128 + lane;
    const int last = 2 * nck - 1;
    auto frag = [&](int st, int i, int part) {
        st = min(st, last);
        const int pr = st >= nck ? 1 : 0;
        return lf[(((int64_t)(2 * pr + i) * nck + st - pr * nck) * 2 + part) * 64];
    };
    uint4 a0h[2], a0l[2], a1h[2], a1l[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        a0h[i] = frag(0, i, 0);
        a0l[i] = frag(0, i, 1);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        a1h[i] = frag(1, i, 0);
        a1l[i] = frag(1, i, 1);
    }
#pragma unroll 1
    for (int pr = 0; pr < 2; ++pr) {
        float4 sv[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int c = 128 * wave + 32 * (2 * pr + i) + 8 * gg + 4 * h;
                sv[i][gg] = *(const float4 *)(sn + c);
            }
        floatx16 ac[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) ac[i][v] = 0.f;
        for (int c = 0; c < nck; c += 2) {   // nck is even: chunk c in set 0, c + 1 in set 1
            const int st = pr * nck + c;
            const uint4 b0h = bh[2 * c], b0l = bl[2 * c];
#pragma unroll
            for (int i = 0; i < 2; ++i) ac[i] = mfma_x3(a0h[i], a0l[i], b0h, b0l, ac[i]);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a0h[i] = frag(st + 2, i, 0);
                a0l[i] = frag(st + 2, i, 1);
            }
            const uint4 b1h = bh[2 * c + 2], b1l = bl[2 * c + 2];
#pragma unroll
            for (int i = 0; i < 2; ++i) ac[i] = mfma_x3(a1h[i], a1l[i], b1h, b1l, ac[i]);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a1h[i] = frag(st + 3, i, 0);
                a1l[i] = frag(st + 3, i, 1);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int c = 128 * wave + 32 * (2 * pr + i) + 8 * gg + 4 * h;
                const float4 v = make_float4(keep ? (ac[i][4 * gg] + sv[i][gg].x) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 1] + sv[i][gg].y) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 2] + sv[i][gg].z) * scale : 0.f,
                                             keep ? (ac[i][4 * gg + 3] + sv[i][gg].w) * scale : 0.f);
                *(float4 *)(base + ((int64_t)(c >> 6) * n + ((c >> 3) & 7)) * n + (c & 7)) = v;
            }
    }
}

}  // namespace

// Split-BF16 fragments of an FP64 operator (rows x cols, row-major, leading dimension lda)
// for the fused kernels: ceil(rows / 32) tiles of nck >= ceil(cols / 16) chunks, 128 uint4
// per tile and chunk (the chunks past the operator's columns zero).
int launch_pack_fragments_x3(const double *A, int rows, int cols, int lda, int nck, uint4 *xf, hipStream_t st) {
    if (nck * 16 < cols) return fail(KIFMM_EINVAL, "split-BF16 operator fragments: too few chunks");
    const int ntile = (rows + 31) / 32;
    const int64_t total = (int64_t)ntile * nck * 64;
    hipLaunchKernelGGL(pack_fragments_x3_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, rows, cols,
                       lda, ntile, nck, xf);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

// chunks of the split-BF16 L2P fragments
int l2p_fragment_chunks_x3(int KD) { return l2p_chunks_x3(KD); }

// Operator fragments for the fused kernels: rows x cols (row-major, leading dimension
// lda) into ceil(rows / 32) tiles of nchunk >= ceil(cols / 8) chunks (the chunks past the
// operator's columns zero).
int launch_pack_fragments(const float *A, int rows, int cols, int lda, int nchunk, float4 *frag, hipStream_t st) {
    if (nchunk * 8 < cols) return fail(KIFMM_EINVAL, "operator fragments: too few chunks");
    const int ntile = (rows + 31) / 32;
    const int64_t total = (int64_t)ntile * nchunk * 64;
    hipLaunchKernelGGL(pack_fragments_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, rows, cols,
                       lda, ntile, nchunk, frag);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

// chunks of the L2P fragments (the fused L2P reads an even number)
int l2p_fragment_chunks(int KD) { return l2p_chunks(KD); }

// The fused kernels apply to FP32 evaluations on leaves of 8^3 cells with at least 4 leaves
// per axis (n % 32 == 0), 16-byte aligned fields, KU % 32 == 0 and KD % 8 == 0, KD <= 256.
bool leafgemm_fits(const Tree &t, int KU, int KD) {
    return t.ell == 8 && t.ellz == 8 && t.R == 1 && t.n % 32 == 0 && t.nb >= 4 && KU % 32 == 0 && KU > 0 && KD % 8 == 0 && KD > 0 &&
           KD <= 256;
}

int run_p2m_permute_in(const Tree &t, const float *I, float vol, const float4 *Af, int KU, float *q, float *cu,
                       hipStream_t st) {
    if ((uintptr_t)I % 16 || (uintptr_t)q % 16 || (uintptr_t)cu % 16) return fail(KIFMM_EINVAL, "fused P2M: misaligned buffer");
    // q may be NULL: the leaf-ordered sources are then not written
    const int64_t nblk = (int64_t)t.nb * t.nb * t.nb / kLeafBlock;
    hipLaunchKernelGGL(p2m_permute_in_kernel, dim3((unsigned)nblk), dim3(256), 0, st, I, t.n, vol, Af, KU / 32, KU, q,
                       cu);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

// the same passes in split BF16 (fragments from launch_pack_fragments_x3)
int run_p2m_permute_in_x3(const Tree &t, const float *I, float vol, const uint4 *Ax, int KU, float *q, float *cu,
                          hipStream_t st) {
    if ((uintptr_t)I % 16 || (uintptr_t)q % 16 || (uintptr_t)cu % 16) return fail(KIFMM_EINVAL, "fused P2M: misaligned buffer");
    const int64_t nblk = (int64_t)t.nb * t.nb * t.nb / kLeafBlock;
    hipLaunchKernelGGL(p2m_permute_in_x3_kernel, dim3((unsigned)nblk), dim3(256), 0, st, I, t.n, vol, Ax, KU / 32, KU,
                       q, cu);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_l2p_permute_out_x3(const Tree &t, const float *cd, int KD, const uint4 *Lx, const float *Snear, float scale,
                           const uint8_t *want, float *S, hipStream_t st) {
    if ((uintptr_t)S % 16 || (uintptr_t)cd % 16 || (uintptr_t)Snear % 16) return fail(KIFMM_EINVAL, "fused L2P: misaligned buffer");
    const int64_t nblk = (int64_t)t.nb * t.nb * t.nb / kLeafBlock;
    hipLaunchKernelGGL(l2p_permute_out_x3_kernel, dim3((unsigned)nblk), dim3(256), 0, st, cd, KD, Lx, Snear, t.n, scale,
                       want, S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_l2p_permute_out(const Tree &t, const float *cd, int KD, const float4 *Lf, const float *Snear, float scale,
                        const uint8_t *want, float *S, hipStream_t st) {
    if ((uintptr_t)S % 16 || (uintptr_t)cd % 16 || (uintptr_t)Snear % 16) return fail(KIFMM_EINVAL, "fused L2P: misaligned buffer");
    const int64_t nblk = (int64_t)t.nb * t.nb * t.nb / kLeafBlock;
    hipLaunchKernelGGL(l2p_permute_out_kernel, dim3((unsigned)nblk), dim3(256), 0, st, cd, KD, Lf, Snear, t.n, scale,
                       want, S);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
