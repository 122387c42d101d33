// The "tap GEMM" engine: every pass of the evaluation is, on a uniform grid, a
// sum over a few taps of one shared dense matrix times the vector of another box:
//
//   out[b][0:M] (+)= sum_t A[op(c, t)] (M x K) . in[src(b, t)][0:K]
//
// for all output boxes b = cls_stride * j + c of a class c.
//   P2M (s2m)   class 0, one tap,  src = b            A = U_u^T G(x^u, leaf cells)
//   M2M (m2m)   class 0, 8 taps,   src = 8 b + child  A = U_u^T G(x^u_P, y^u_child) V_u S^-1
//   M2L (m2l)   8 parity classes, 189 taps, src = b + offset (Morton neighbour)
//   L2L (l2l)   8 child classes, one tap, src = b >> 3
//   L2P         class 0, one tap,  src = b            A = G(leaf cells, y^d) V_d S^-1
//   P2P         class 0, 27 taps,  src = neighbour leaf, A = near-range matrix
// Boxes outside the grid contribute nothing (their src is -1 and loads zeros).
//
// Work split: a workgroup owns an output tile (BM rows x 64 boxes of one class)
// and a group of taps.  Tiles are numbered with the row tile fastest, and each
// XCD takes a contiguous range of tile numbers, so the workgroups resident on one
// XCD share the source boxes of a compact region in its L2.  When the tap list is
// split over G groups (to put enough workgroups on the 256 CUs at coarse levels)
// each group writes an FP32 partial sum to scratch and reduce_partials adds the
// groups in a fixed order in FP64, so results do not depend on scheduling.
//
// Kernels:
//   tapgemm_f32_staged      FP32 on v_mfma_f32_32x32x2f32, operators of more than
//                           64 rows (128-row tiles)
//   tapgemm_lp_staged<TL,NP> BF16 or FP16 operands on v_mfma_f32_32x32x16_{bf16,f16}
//                           with FP32 accumulation.  The input is split beforehand
//                           by split_lp_kernel: v = in / max|in|, B_hi = round(v),
//                           B_lo = round(v - B_hi); operators are stored split the
//                           same way.  NP = 1: A_hi B_hi; NP = 3: A_hi B_hi +
//                           A_hi B_lo + A_lo B_hi (about 16 mantissa bits)
//   tapgemm_f32_small       FP32 on v_mfma_f32_16x16x4f32, 64-row tiles
//   tapgemm_lp<TL,X3>       low precision for small operators and for inputs that
//                           are not split beforehand: the input is scaled and
//                           rounded while it is staged through registers
//   tapgemm_valu<T>         LDS-tiled VALU version for FP64 (and any T)
//
// The staged kernels copy operand tiles from global memory straight into LDS
// (global_load_lds_dwordx4), three chunks deep: while chunk c is multiplied, the
// copies of chunks c+1 and c+2 are in flight, and one barrier per chunk hands a
// stage from the copies to the readers.  Each thread's copies land at fixed
// 16-byte positions; the global address a position is filled from is chosen so
// that the tile ends up in an XOR-swizzled layout that the MFMA fragment reads
// see without bank conflicts.
//
// Inside a 32-wide K chunk the reduction index is permuted so that one 16-byte
// LDS read feeds several MFMA steps (products are summed in any order, so A and B
// only have to use the same permutation).  MFMA partial sums are folded into FP64
// totals every few chunks (at most 96 products per FP32 chain), so long near-field
// and M2L sums keep the rounding of one short chain.
#include "common.h"
#include "tapgemm.h"

#include <type_traits>
#include <utility>

namespace kifmm {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// zr <= 1: b = sample * nl^3 + morton(x, y, z), neighbours stay inside the sample (the
// surrogate's batches, or the single cube of the tree).  zr > 1: the level is a column of
// zr cubes of nl^3 boxes stacked along z (a tree over a box of zr cubes), b = root *
// nl^3 + morton(x, y, z - root nl), and neighbours cross from one cube into the next.
__device__ inline int64_t source_box(int mode, int64_t b, int off, int nl, int zr = 1) {
    switch (mode) {
        case SRC_SAME: return b;
        case SRC_CHILD: return 8 * b + off;
        case SRC_PARENT: return b >> 3;
        default: {
            int lg = 0;
            while ((1 << lg) < nl) ++lg;
            const int64_t root = b >> (3 * lg);
            int x, y, z;
            morton_decode((uint32_t)(b - (root << (3 * lg))), x, y, z);
            x += ((off >> 10) & 31) - 16;
            y += ((off >> 5) & 31) - 16;
            z += (off & 31) - 16;
            if (zr <= 1) {
                if (x < 0 || y < 0 || z < 0 || x >= nl || y >= nl || z >= nl) return -1;
                return (root << (3 * lg)) + (int64_t)morton_encode(x, y, z);
            }
            const int64_t zg = root * nl + z;   // z in the column
            if (x < 0 || y < 0 || zg < 0 || x >= nl || y >= nl || zg >= (int64_t)zr * nl) return -1;
            return ((zg >> lg) << (3 * lg)) + (int64_t)morton_encode(x, y, (uint32_t)(zg & (nl - 1)));
        }
    }
}

__device__ inline int tap_op_of(const int *tab, const int *inl, int i) { return tab ? tab[i] : inl[i]; }

constexpr int BN = 64;     // boxes per tile

// Workgroups are dispatched round-robin over the 8 XCDs (linear id % 8), and each XCD
// has its own L2.  Tile index of this workgroup: XCD x gets the contiguous range
// [x * nt / 8, (x + 1) * nt / 8) of the Morton-ordered box tiles, a spatially compact
// region, so the neighbour halos and operator tiles it reads are shared in one L2.
__device__ inline int64_t xcd_tile(int64_t bx, int64_t nt) {
    if (nt % 8 != 0) return bx;
    return (bx % 8) * (nt / 8) + bx / 8;
}

// Tile of block bx for launches that skip work by box flags (zero sources, unwanted
// targets): the skipped tiles cluster in Morton ranges, so one contiguous eighth per XCD
// could leave most XCDs idle.  Each XCD takes every 8th run of 8 box tiles (rt row tiles
// each) instead, which keeps neighbouring boxes in one L2 and spreads the work.
__device__ inline int64_t sparse_tile(int64_t bx, int64_t nt, int rt) {
    const int64_t run = 8 * (int64_t)rt;
    if (nt % (8 * run) != 0) return bx;
    const int64_t k = bx % 8, i = bx / 8;
    return ((i / run) * 8 + k) * run + i % run;
}
constexpr int BK = 32;     // reduction chunk
constexpr int APAD = 4;    // LDS row padding (floats)

__device__ inline float comp(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// s_waitcnt immediate: at most `vm` vector-memory operations outstanding, no LDS/scalar
// operation outstanding (expcnt left free)
constexpr int waitcnt_vm_lgkm0(int vm) { return (vm & 15) | ((vm >> 4) << 14) | 0x70; }

// Workgroup barrier.  The memory clobber keeps the compiler from moving loads or stores
// across it; each wave has already waited for its own LDS reads and for its own
// asynchronous global-to-LDS copies with s_waitcnt.
__device__ inline void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

__device__ __align__(16) float kZeroChunk[BK];   // zero source for boxes outside the grid

// asynchronous copy of 16 bytes per lane from global memory to LDS: lane l writes
// lds + 16 l (lds is the same for the whole wave)
__device__ inline void copy16_to_lds(const float *g, float *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0); }

// Swizzled position of the 16-byte group kq (0..7) of row r in a BK = 32 float tile:
// 16 consecutive rows read at one kq hit 16 distinct 16-byte bank groups.
__device__ inline int swz_slot(int r, int kq) { return r * 8 + (kq ^ ((r ^ (r >> 3)) & 7)); }

// Twelve 16-byte LDS reads (byte addresses a[i]) completed before returning.  Written
// as one asm block so that the compiler, which cannot tell these reads from the
// asynchronous copies still in flight into other stages, adds no wait for them.
__device__ inline void lds_read12(const int (&a)[12], float4 (&v)[12]) {
    asm volatile(
        "ds_read_b128 %0, %12\n"
        "ds_read_b128 %1, %13\n"
        "ds_read_b128 %2, %14\n"
        "ds_read_b128 %3, %15\n"
        "ds_read_b128 %4, %16\n"
        "ds_read_b128 %5, %17\n"
        "ds_read_b128 %6, %18\n"
        "ds_read_b128 %7, %19\n"
        "ds_read_b128 %8, %20\n"
        "ds_read_b128 %9, %21\n"
        "ds_read_b128 %10, %22\n"
        "ds_read_b128 %11, %23\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
          "=&v"(v[6]), "=&v"(v[7]), "=&v"(v[8]), "=&v"(v[9]), "=&v"(v[10]), "=&v"(v[11])
        : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]),
          "v"(a[6]), "v"(a[7]), "v"(a[8]), "v"(a[9]), "v"(a[10]), "v"(a[11])
        : "memory");
}

// FP32 tap GEMM for operators of at most 64 rows: 64 x 64 tiles on v_mfma_f32_16x16x4f32,
// operands staged through registers into padded LDS tiles.
template <int PASS>
__global__ __launch_bounds__(256) void tapgemm_f32_small(TapArgs<float, float, float> p) {
    constexpr int BM = 64;
    constexpr int IM = BM / 32;          // 16-row blocks per wave (waves: 2 x 2)
    constexpr int JN = 2;                // 16-box blocks per wave
    constexpr int AR = BM / 32;          // float4 loads of A per thread per chunk
    __shared__ float As[BM][BK + APAD];
    __shared__ float Bs[BN][BK + APAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = p.groups;
    const int cls = blockIdx.z / G, grp = blockIdx.z % G;
    const int tpg = (p.ntaps + G - 1) / G;
    const int t0 = grp * tpg, t1 = min(p.ntaps, t0 + tpg);
    const int RT = (p.M + BM - 1) / BM;                 // row tiles: the fastest tile index
    const int64_t lin = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t j0 = lin / RT * BN;
    const int m0 = (int)(lin % RT) * BM;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
    const int KC = p.K / BK;
    const int total = t1 > t0 ? (t1 - t0) * KC : 0;

    floatx4 acc[IM][JN];
    double tot[IM][JN][4];
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) {
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[i][j][v] = 0.0;
        }

    // loader: rows r*32 + tid/8, k = (tid%8)*4 .. +3 of the chunk
    const int lrow = tid >> 3, lk = (tid & 7) * 4;
    float4 ra[AR], rb[2];
    int64_t lsrc[2] = {-1, -1};
    const float *Aop = p.A;
    auto load = [&](int it) {
        const int t = t0 + it / KC, kc = it % KC;
        if (kc == 0) {
            const int op = tap_op_of(p.tap_op, p.inl_op, cls * p.ntaps + t);
            const int off = tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t);
            Aop = p.A + (int64_t)op * p.a_stride;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int64_t j = j0 + r * 32 + lrow;
                lsrc[r] = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
            }
        }
        const int k = kc * BK + lk;
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int row = m0 + r * 32 + lrow;
            ra[r] = row < p.M ? *(const float4 *)(Aop + (int64_t)row * p.K + k) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
            rb[r] = lsrc[r] >= 0 ? *(const float4 *)(p.in + lsrc[r] * p.in_ld + k) : make_float4(0.f, 0.f, 0.f, 0.f);
    };

    if (total > 0) load(0);
    const int q = lane >> 4, c16 = lane & 15;
    for (int it = 0; it < total; ++it) {
        __syncthreads();   // the previous chunk's fragments have been read
#pragma unroll
        for (int r = 0; r < AR; ++r) *(float4 *)&As[r * 32 + lrow][lk] = ra[r];
#pragma unroll
        for (int r = 0; r < 2; ++r) *(float4 *)&Bs[r * 32 + lrow][lk] = rb[r];
        __syncthreads();
        if (it + 1 < total) load(it + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // k = 8q + 4h .. 8q + 4h + 3
            float4 af[IM], bfr[JN];
#pragma unroll
            for (int i = 0; i < IM; ++i) af[i] = *(const float4 *)&As[wr + 16 * i + c16][8 * q + 4 * h];
#pragma unroll
            for (int j = 0; j < JN; ++j) bfr[j] = *(const float4 *)&Bs[wc + 16 * j + c16][8 * q + 4 * h];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < IM; ++i)
#pragma unroll
                    for (int j = 0; j < JN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(comp(af[i], e), comp(bfr[j], e),
                                                                        acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
#pragma unroll
                for (int v = 0; v < 4; ++v) tot[i][j][v] += (double)acc[i][j][v];
                acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    }
    // D layout of 16x16x4: lane holds rows 4*(lane/16)+v, column lane%16
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int jj = 0; jj < JN; ++jj) {
            const int row = m0 + wr + 16 * i + 4 * (lane >> 4);
            const int64_t j = j0 + wc + 16 * jj + (lane & 15);
            if (row < p.M && j < p.n_per_class) {
                const int64_t b = (int64_t)p.cls_stride * j + cls;
                double v0 = tot[i][jj][0], v1 = tot[i][jj][1], v2 = tot[i][jj][2], v3 = tot[i][jj][3];
                float *o;
                if (G > 1) {
                    o = p.part + ((int64_t)grp * p.n_boxes + b) * p.out_ld + row;
                } else {
                    o = p.out + b * p.out_ld + row;
                    if (p.accumulate) {
                        const float4 old = *(const float4 *)o;
                        v0 += old.x; v1 += old.y; v2 += old.z; v3 += old.w;
                    }
                }
                *(float4 *)o = make_float4((float)v0, (float)v1, (float)v2, (float)v3);
            }
        }
}

// Taps of this workgroup's group [t0, t1) whose source boxes are not all zero for the 64
// output boxes j0 .. j0+63 of class cls (every tap when p.in_nz is null).  Returns the
// count and leaves, in increasing order, the offsets t - t0 of those taps in lane i of
// act[r] for the (64 r + i)-th of them.  A skipped tap adds exact zeros, so the sum over
// the remaining taps is the same sum.  None of the taps is kept when p.out_need marks
// none of the 64 output boxes as wanted.  Called by all 256 threads; uses flags[256].
template <typename TA, typename TI, typename TO>
__device__ inline int active_taps(const TapArgs<TA, TI, TO> &p, int cls, int t0, int t1, int64_t j0,
                                  uint8_t *flags, int (&act)[4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nt = t1 - t0;
    if (p.out_need) {   // every wave takes the same ballot, so all return together or none
        const int64_t j = j0 + lane;
        const bool want = j < p.n_per_class && p.out_need[(int64_t)p.cls_stride * j + cls] != 0;
        if (__ballot(want) == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) act[r] = 0;
            return 0;
        }
    }
    if (!p.in_nz) {
#pragma unroll
        for (int r = 0; r < 4; ++r) act[r] = 64 * r + lane;
        return nt > 0 ? nt : 0;
    }
    for (int t = t0 + wave; t < t1; t += 4) {   // one wave per tap, one lane per box
        const int off = tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t);
        const int64_t j = j0 + lane;
        const int64_t src = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
        const bool live = src >= 0 && p.in_nz[src] != 0;
        const uint64_t any = __ballot(live);
        if (lane == 0) flags[t - t0] = any != 0;
    }
    __syncthreads();
    // compaction, computed the same way in every wave: four 64-tap ballots, then lane L of
    // act[r] looks up the set flag of rank 64 r + L
    uint64_t m[4];
    int cum[5];
    cum[0] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int t = 64 * c + lane;
        m[c] = __ballot(t < nt && flags[t] != 0);
        cum[c + 1] = cum[c] + __popcll(m[c]);
    }
    const int count = cum[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 64 * r + lane;
        act[r] = 0;
        if (k < count) {
            const int c = (k >= cum[1]) + (k >= cum[2]) + (k >= cum[3]);
            const int want = k - (c == 0 ? 0 : c == 1 ? cum[1] : c == 2 ? cum[2] : cum[3]);
            const uint64_t mm = c == 0 ? m[0] : c == 1 ? m[1] : c == 2 ? m[2] : m[3];
            int lo = 0, hi = 63;   // position of the set bit of rank `want` in mm
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (__popcll(mm & ((2ull << mid) - 1ull)) > want) hi = mid;
                else lo = mid + 1;
            }
            act[r] = 64 * c + lo;
        }
    }
    __syncthreads();   // flags may be reused
    return count;
}

// Calls f(integral_constant<int, U>) for U = 0, 1, ... in order while it returns true.
template <class F, int... U>
__device__ inline void unrolled_steps(F &f, std::integer_sequence<int, U...>) {
    (f(std::integral_constant<int, U>()) && ...);
}

// Waits until at most n * per vector-memory operations are outstanding (0 <= n <= 4),
// with no LDS or scalar operation outstanding, then joins the workgroup barrier.
template <int PER>
__device__ inline void wait_outstanding_then_barrier(int n) {
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0)); break;
        case 1: __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(PER)); break;
        case 2: __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(2 * PER)); break;
        case 3: __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(3 * PER)); break;
        default: __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(4 * PER)); break;
    }
    lds_barrier();
}

// FP32 tap GEMM on v_mfma_f32_32x32x2f32, BM = 128 rows x 64 boxes per workgroup, each
// wave a 64 x 32 tile.  Operand tiles are copied from global memory straight into LDS
// (global_load_lds_dwordx4) three stages deep: two chunks of copies are in flight while
// the third chunk is multiplied.
template <int PASS>
__global__ __launch_bounds__(256) void tapgemm_f32_staged(TapArgs<float, float, float> p) {
    constexpr int BM = 128;
    constexpr int IM = 2;                    // 32-row blocks per wave (waves: 2 x 2)
    constexpr int AR = BM * 8 / 256;         // 16-byte copies of A per thread per chunk
    constexpr int BR = BN * 8 / 256;         // 16-byte copies of B per thread per chunk
    constexpr int LPC = AR + BR;
    constexpr int STG = (BM + BN) * BK;      // floats per stage: A tile then B tile
    __shared__ __align__(16) float St[3 * STG];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = p.groups;
    const int cls = blockIdx.z / G, grp = blockIdx.z % G;
    const int tpg = (p.ntaps + G - 1) / G;
    const int t0 = grp * tpg, t1 = min(p.ntaps, t0 + tpg);
    const int RT = (p.M + BM - 1) / BM;                 // row tiles: the fastest tile index
    const int64_t lin = p.in_nz || p.out_need ? sparse_tile(blockIdx.x, gridDim.x, RT)
                                              : xcd_tile(blockIdx.x, gridDim.x);
    const int64_t j0 = lin / RT * BN;
    const int m0 = (int)(lin % RT) * BM;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
    const int KC = p.K / BK;
    __shared__ uint8_t tap_flags[256];
    int act[4];
    const int nact = active_taps(p, cls, t0, t1, j0, tap_flags, act);   // taps with nonzero sources
    const int total = nact * KC;

    floatx16 acc[IM];
    double tot[IM][16];
#pragma unroll
    for (int i = 0; i < IM; ++i) {
#pragma unroll
        for (int v = 0; v < 16; ++v) { acc[i][v] = 0.f; tot[i][v] = 0.0; }
    }

    // this group's live taps: lane i of register r holds the (64 r + i)-th (read with readlane)
    int my_op[4], my_off[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = t0 + act[r];
        const bool live = 64 * r + lane < nact;
        my_op[r] = live ? tap_op_of(p.tap_op, p.inl_op, cls * p.ntaps + t) : 0;
        my_off[r] = live ? tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t) : 0;
    }

    // copy r of this thread fills 16-byte position (r * 4 + wave) * 64 + lane of a tile
    int a_off[AR], b_kq[BR];
#pragma unroll
    for (int r = 0; r < AR; ++r) {
        const int pos = (r * 4 + wave) * 64 + lane, row = pos >> 3;
        const int kq = (pos & 7) ^ ((row ^ (row >> 3)) & 7);
        a_off[r] = min(m0 + row, p.M - 1) * p.K + kq * 4;   // rows past M are never stored
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const int pos = (r * 4 + wave) * 64 + lane, box = pos >> 3;
        b_kq[r] = (pos & 7) ^ ((box ^ (box >> 3)) & 7);
    }
    const float *bsrc[BR];
    const float *Aop = p.A;
    auto issue = [&](int it, int stage) {
        const int tt = it / KC, kc = it % KC;
        if (kc == 0) {
            int op = 0, off = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if ((tt >> 6) == r) {
                    op = __builtin_amdgcn_readlane(my_op[r], tt & 63);
                    off = __builtin_amdgcn_readlane(my_off[r], tt & 63);
                }
            Aop = p.A + (int64_t)op * p.a_stride;
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const int64_t j = j0 + (r * 4 + wave) * 8 + (lane >> 3);
                const int64_t src = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
                bsrc[r] = src >= 0 ? p.in + src * p.in_ld : nullptr;
            }
        }
        const int k = kc * BK;
        float *As = St + stage * STG, *Bs = As + BM * BK;
#pragma unroll
        for (int r = 0; r < AR; ++r) copy16_to_lds(Aop + a_off[r] + k, As + (r * 4 + wave) * 256);
#pragma unroll
        for (int r = 0; r < BR; ++r)
            copy16_to_lds(bsrc[r] ? bsrc[r] + k + b_kq[r] * 4 : kZeroChunk + b_kq[r] * 4, Bs + (r * 4 + wave) * 256);
    };

    // LDS byte addresses (stage 0) of this lane's fragments: for h = 0..3, the A rows of
    // blocks 0 and 1 and the B column, at k = 16q + 4h .. 16q + 4h + 3
    const int q = lane >> 5, r32 = lane & 31;
    int fa[12];
    {
        const int base = (int)(uintptr_t)(__attribute__((address_space(3))) float *)St;   // LDS byte address
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int kq = 4 * q + h;
            fa[3 * h] = base + swz_slot(wr + r32, kq) * 16;
            fa[3 * h + 1] = base + swz_slot(wr + 32 + r32, kq) * 16;
            fa[3 * h + 2] = base + BM * BK * 4 + swz_slot(wc + r32, kq) * 16;
        }
    }
    auto compute = [&](const float4 (&fr)[12]) {
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < IM; ++i)
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(comp(fr[3 * h + i], e), comp(fr[3 * h + 2], e), acc[i],
                                                                0, 0, 0);
    };
    auto fold = [&]() {   // FP64 totals take the FP32 partial sums of the last NS chunks
#pragma unroll
        for (int i = 0; i < IM; ++i) {
#pragma unroll
            for (int v = 0; v < 16; ++v) { tot[i][v] += (double)acc[i][v]; acc[i][v] = 0.f; }
        }
    };
    constexpr int NS = 3;
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
        if (u < total) issue(u, u);
    float4 fr[12];
    int it = 0;
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        const int c = it + u;
        if (c >= total) return false;
        wait_outstanding_then_barrier<LPC>(min(total - 1 - c, NS - 2));
        int a[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) a[i] = fa[i] + u * STG * 4;
        lds_read12(a, fr);
        if (c + NS - 1 < total) issue(c + NS - 1, (u + NS - 1) % NS);
        compute(fr);
        return true;
    };
    for (; it < total; it += NS) {
        unrolled_steps(step, std::make_integer_sequence<int, NS>());
        fold();
    }
    // D layout of 32x32x2: lane holds column lane%32 and, in registers 4g .. 4g+3,
    // rows 8g + 4*(lane/32) + 0..3
    const int64_t j = j0 + wc + r32;
    if (j < p.n_per_class) {
        const int64_t b = (int64_t)p.cls_stride * j + cls;
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int row = m0 + wr + 32 * i + 8 * g + 4 * q;
                if (row < p.M) {
                    double v0 = tot[i][4 * g], v1 = tot[i][4 * g + 1], v2 = tot[i][4 * g + 2], v3 = tot[i][4 * g + 3];
                    float *o;
                    if (G > 1) {
                        o = p.part + ((int64_t)grp * p.n_boxes + b) * p.out_ld + row;
                    } else {
                        o = p.out + b * p.out_ld + row;
                        if (p.accumulate) {
                            const float4 old = *(const float4 *)o;
                            v0 += old.x; v1 += old.y; v2 += old.z; v3 += old.w;
                        }
                    }
                    *(float4 *)o = make_float4((float)v0, (float)v1, (float)v2, (float)v3);
                }
            }
    }
}

// out[e] = (accumulate ? out[e] : 0) + sum_g part[g][e], FP64 sum in g order
__global__ void reduce_partials(const float *__restrict__ part, int G, int64_t n, int accumulate,
                                float *__restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double s = accumulate ? (double)out[e] : 0.0;
        for (int g = 0; g < G; ++g) s += (double)part[(int64_t)g * n + e];
        out[e] = (float)s;
    }
}

// ------------------------------------------------------- low precision ----
template <typename TL> struct LPVec;
template <> struct LPVec<__bf16> { typedef bf16x8 type; };
template <> struct LPVec<_Float16> { typedef halfx8 type; };

template <typename TL>
__device__ inline floatx4 mfma_lp(const typename LPVec<TL>::type &a, const typename LPVec<TL>::type &b, floatx4 c) {
    if constexpr (std::is_same<TL, __bf16>::value) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

constexpr int LBK = 32, LPAD = 8;

// BM = 128 rows x 64 boxes; per 32-wide chunk one MFMA step per block (x3 for split BF16)
template <typename TL, bool X3, int PASS, int BM>
__global__ __launch_bounds__(256) void tapgemm_lp(TapArgs<TL, float, float> p) {
    typedef typename LPVec<TL>::type vec8;
    constexpr int IM = BM / 32, JN = 2, NA = X3 ? 2 : 1;
    constexpr int AR = BM >= 64 ? BM / 64 : 1;   // A row passes of the loader (64 rows each)
    __shared__ TL As[NA][BM][LBK + LPAD];
    __shared__ TL Bs[NA][BN][LBK + LPAD];
    __shared__ float in_scale_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = p.groups;
    const int cls = blockIdx.z / G, grp = blockIdx.z % G;
    const int tpg = (p.ntaps + G - 1) / G;
    const int t0 = grp * tpg, t1 = min(p.ntaps, t0 + tpg);
    const int RT = (p.M + BM - 1) / BM;                 // row tiles: the fastest tile index
    const int64_t lin = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t j0 = lin / RT * BN;
    const int m0 = (int)(lin % RT) * BM;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
    const int KC = p.K / LBK;
    const int total = t1 > t0 ? (t1 - t0) * KC : 0;
    if (tid == 0) {
        float mx = 0.f;
        for (int i = 0; i < p.n_amax; ++i) mx = fmaxf(mx, p.amax[i]);
        in_scale_sh = mx > 0.f ? 1.0f / mx : 1.0f;
    }
    floatx4 acc[IM][JN];
    double tot[IM][JN][4];
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) {
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[i][j][v] = 0.0;
        }
    __syncthreads();
    const float sin = in_scale_sh;
    // loader: A rows r*64 + tid/4 (8 values at k = (tid%4)*8); B box tid/4
    const int lrow = tid >> 2, lk = (tid & 3) * 8;
    vec8 ra[AR][NA], rb[NA];
    int64_t lsrc = -1;
    const TL *Ahi = p.A, *Alo = p.A2;
    auto load = [&](int it) {
        const int t = t0 + it / KC, kc = it % KC;
        if (kc == 0) {
            const int op = tap_op_of(p.tap_op, p.inl_op, cls * p.ntaps + t);
            const int off = tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t);
            Ahi = p.A + (int64_t)op * p.a_stride;
            if (X3) Alo = p.A2 + (int64_t)op * p.a_stride;
            const int64_t j = j0 + lrow;
            lsrc = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
        }
        const int k = kc * LBK + lk;
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int row = m0 + r * 64 + lrow;
            if (row < p.M && r * 64 + lrow < BM) {
                ra[r][0] = *(const vec8 *)(Ahi + (int64_t)row * p.K + k);
                if (X3) ra[r][NA - 1] = *(const vec8 *)(Alo + (int64_t)row * p.K + k);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    ra[r][0][e] = (TL)0.f;
                    ra[r][NA - 1][e] = (TL)0.f;
                }
            }
        }
        if (lsrc >= 0) {
            const float4 x0 = *(const float4 *)(p.in + lsrc * p.in_ld + k);
            const float4 x1 = *(const float4 *)(p.in + lsrc * p.in_ld + k + 4);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = (e < 4 ? comp(x0, e) : comp(x1, e - 4)) * sin;
                const TL hi = (TL)v;
                rb[0][e] = hi;
                if (X3) rb[NA - 1][e] = (TL)(v - (float)hi);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                rb[0][e] = (TL)0.f;
                rb[NA - 1][e] = (TL)0.f;
            }
        }
    };
    if (total > 0) load(0);
    const int kl = 8 * (lane >> 4), c16 = lane & 15;
    for (int it = 0; it < total; ++it) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NA; ++h) {
#pragma unroll
            for (int r = 0; r < AR; ++r)
                if (r * 64 + lrow < BM) *(vec8 *)&As[h][r * 64 + lrow][lk] = ra[r][h];
            *(vec8 *)&Bs[h][lrow][lk] = rb[h];
        }
        __syncthreads();
        if (it + 1 < total) load(it + 1);
        vec8 af[NA][IM], bfr[NA][JN];
#pragma unroll
        for (int h = 0; h < NA; ++h) {
#pragma unroll
            for (int i = 0; i < IM; ++i) af[h][i] = *(const vec8 *)&As[h][wr + 16 * i + c16][kl];
#pragma unroll
            for (int j = 0; j < JN; ++j) bfr[h][j] = *(const vec8 *)&Bs[h][wc + 16 * j + c16][kl];
        }
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
                acc[i][j] = mfma_lp<TL>(af[0][i], bfr[0][j], acc[i][j]);
                if (X3) {
                    acc[i][j] = mfma_lp<TL>(af[0][i], bfr[NA - 1][j], acc[i][j]);
                    acc[i][j] = mfma_lp<TL>(af[NA - 1][i], bfr[0][j], acc[i][j]);
                }
            }
        if ((it & 3) == 3 || it + 1 == total) {
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int j = 0; j < JN; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) tot[i][j][v] += (double)acc[i][j][v];
                    acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
        }
    }
    const double oscale = (double)p.op_scale / (double)sin;
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int jj = 0; jj < JN; ++jj) {
            const int row = m0 + wr + 16 * i + 4 * (lane >> 4);
            const int64_t j = j0 + wc + 16 * jj + (lane & 15);
            if (row < p.M && j < p.n_per_class) {
                const int64_t b = (int64_t)p.cls_stride * j + cls;
                double v0 = tot[i][jj][0] * oscale, v1 = tot[i][jj][1] * oscale;
                double v2 = tot[i][jj][2] * oscale, v3 = tot[i][jj][3] * oscale;
                float *o;
                if (G > 1) {
                    o = p.part + ((int64_t)grp * p.n_boxes + b) * p.out_ld + row;
                } else {
                    o = p.out + b * p.out_ld + row;
                    if (p.accumulate) {
                        const float4 old = *(const float4 *)o;
                        v0 += old.x; v1 += old.y; v2 += old.z; v3 += old.w;
                    }
                }
                *(float4 *)o = make_float4((float)v0, (float)v1, (float)v2, (float)v3);
            }
        }
}

// Generic LDS-tiled VALU version: 64 rows x 32 boxes per workgroup, each thread
// 4 rows x 2 boxes.  No tap split.
constexpr int VM = 64, VN = 32, VK = 16;
template <typename T>
__global__ __launch_bounds__(256) void tapgemm_valu(TapArgs<T, T, T> p) {
    __shared__ T As[VK][VM + 1];
    __shared__ T Bs[VK][VN + 1];
    __shared__ int64_t srcs[VN];
    const int cls = blockIdx.z;
    const int64_t j0 = (int64_t)blockIdx.x * VN;
    const int m0 = blockIdx.y * VM;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    T acc[4][2] = {};
    for (int t = 0; t < p.ntaps; ++t) {
        const int op = tap_op_of(p.tap_op, p.inl_op, cls * p.ntaps + t);
        const int off = tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t);
        __syncthreads();
        if (tid < VN) {
            const int64_t j = j0 + tid;
            srcs[tid] = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
        }
        __syncthreads();
        const T *Aop = p.A + (int64_t)op * p.a_stride;
        for (int k0 = 0; k0 < p.K; k0 += VK) {
            for (int e = tid; e < VM * VK; e += 256) {
                const int r = e / VK, kk = e % VK;
                As[kk][r] = (m0 + r < p.M && k0 + kk < p.K) ? Aop[(int64_t)(m0 + r) * p.K + k0 + kk] : T(0);
            }
            for (int e = tid; e < VN * VK; e += 256) {
                const int c = e / VK, kk = e % VK;
                const int64_t s = srcs[c];
                Bs[kk][c] = (s >= 0 && k0 + kk < p.K) ? p.in[s * p.in_ld + k0 + kk] : T(0);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < VK; ++kk) {
                T a[4], b[2];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) b[jj] = Bs[kk][tx + 16 * jj];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = fma(a[i], b[jj], acc[i][jj]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int row = m0 + ty + 16 * i;
            const int64_t j = j0 + tx + 16 * jj;
            if (row < p.M && j < p.n_per_class) {
                const int64_t b = (int64_t)p.cls_stride * j + cls;
                T *o = p.out + b * p.out_ld + row;
                *o = p.accumulate ? *o + acc[i][jj] : acc[i][jj];
            }
        }
}

// ----------------------------------------------------------- weight gradient ----
// dW[t] (M x K) = sum_j dY[b_j] X[src_j]^T: a GEMM whose reduction runs over voxels.
// Workgroup = one tap, one BW x BW tile of dW, one group of voxels; voxels are staged
// 32 at a time, transposed into LDS (reduction index innermost), operands rounded to
// TL (FP32 or BF16) and multiplied on MFMA with FP32 accumulation and FP64 folding.
// Voxel groups write partials that reduce_partials adds in a fixed order.
template <typename TL, int BW>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs p) {
    constexpr int WK = 32, PAD = std::is_same<TL, float>::value ? 4 : 8;
    constexpr int CPT = BW / 8;                 // channels per loader thread
    constexpr int IMW = BW / 32;                // 16-blocks per wave per dimension
    __shared__ TL As[BW][WK + PAD];
    __shared__ TL Bs[BW][WK + PAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t = blockIdx.z, g = blockIdx.x;
    const int tilesK = p.K / BW;
    const int m0 = (blockIdx.y / tilesK) * BW, k0 = (blockIdx.y % tilesK) * BW;
    const int cls = p.class_is_tap ? t : 0;
    const int off = p.tap_off[t];
    int64_t per = (p.n_per_class + p.groups - 1) / p.groups;
    per = (per + WK - 1) / WK * WK;
    const int64_t ja = (int64_t)g * per, jb = min(p.n_per_class, ja + per);
    const int wr = (wave >> 1) * (BW / 2), wc = (wave & 1) * (BW / 2);
    floatx4 acc[IMW][IMW];
    double tot[IMW][IMW][4];
#pragma unroll
    for (int i = 0; i < IMW; ++i)
#pragma unroll
        for (int j = 0; j < IMW; ++j) {
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[i][j][v] = 0.0;
        }
    const int kk = tid >> 3, cg = (tid & 7) * CPT;
    const int q = lane >> 4, c16 = lane & 15;
    int nchunk = 0;
    for (int64_t j0 = ja; j0 < jb; j0 += WK, ++nchunk) {
        float dv[CPT], xv[CPT];
        const int64_t j = j0 + kk;
#pragma unroll
        for (int e = 0; e < CPT; ++e) { dv[e] = 0.f; xv[e] = 0.f; }
        if (j < jb) {
            const int64_t b = (int64_t)p.cls_stride * j + cls;
            const int64_t src = source_box(p.mode, b, off, p.nl);
#pragma unroll
            for (int e = 0; e < CPT; e += 4) {
                const float4 a = *(const float4 *)(p.dy + b * p.M + m0 + cg + e);
                dv[e] = a.x; dv[e + 1] = a.y; dv[e + 2] = a.z; dv[e + 3] = a.w;
            }
            if (src >= 0) {
#pragma unroll
                for (int e = 0; e < CPT; e += 4) {
                    const float4 a = *(const float4 *)(p.x + src * p.K + k0 + cg + e);
                    xv[e] = a.x; xv[e + 1] = a.y; xv[e + 2] = a.z; xv[e + 3] = a.w;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            As[cg + e][kk] = (TL)dv[e];
            Bs[cg + e][kk] = (TL)xv[e];
        }
        __syncthreads();
        if constexpr (std::is_same<TL, float>::value) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float4 af[IMW], bfr[IMW];
#pragma unroll
                for (int i = 0; i < IMW; ++i) {
                    af[i] = *(const float4 *)&As[wr + 16 * i + c16][8 * q + 4 * h];
                    bfr[i] = *(const float4 *)&Bs[wc + 16 * i + c16][8 * q + 4 * h];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int i = 0; i < IMW; ++i)
#pragma unroll
                        for (int jj = 0; jj < IMW; ++jj)
                            acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(comp(af[i], e), comp(bfr[jj], e),
                                                                             acc[i][jj], 0, 0, 0);
            }
        } else {
            bf16x8 af[IMW], bfr[IMW];
#pragma unroll
            for (int i = 0; i < IMW; ++i) {
                af[i] = *(const bf16x8 *)&As[wr + 16 * i + c16][8 * q];
                bfr[i] = *(const bf16x8 *)&Bs[wc + 16 * i + c16][8 * q];
            }
#pragma unroll
            for (int i = 0; i < IMW; ++i)
#pragma unroll
                for (int jj = 0; jj < IMW; ++jj)
                    acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[jj], acc[i][jj], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < IMW; ++i)
#pragma unroll
            for (int jj = 0; jj < IMW; ++jj) {
#pragma unroll
                for (int v = 0; v < 4; ++v) tot[i][jj][v] += (double)acc[i][jj][v];
                acc[i][jj] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    }
    float *out = p.groups > 1 ? p.part + ((int64_t)g * p.ntaps + t) * p.M * p.K
                              : p.dw + (int64_t)t * p.M * p.K;
#pragma unroll
    for (int i = 0; i < IMW; ++i)
#pragma unroll
        for (int jj = 0; jj < IMW; ++jj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wr + 16 * i + 4 * (lane >> 4) + v;
                const int col = k0 + wc + 16 * jj + (lane & 15);
                out[(int64_t)row * p.K + col] = (float)tot[i][jj][v];
            }
}

// per-block partial max |x| over n values (for the low-precision input scale)
__global__ void amax_partial(const float *__restrict__ x, int64_t n, float *__restrict__ part) {
    __shared__ float sh[4];
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// ------------------------------------------------- staged low precision ----
// Input split for the staged kernel: v = x / max|x|, hi = round(v), lo = round(v - hi).
template <typename TL>
__global__ void split_lp_kernel(const float *__restrict__ x, int64_t n, const float *__restrict__ amax, int n_amax,
                                TL *__restrict__ hi, TL *__restrict__ lo) {
    __shared__ float s_sh;
    if (threadIdx.x == 0) {
        float mx = 0.f;
        for (int i = 0; i < n_amax; ++i) mx = fmaxf(mx, amax[i]);
        s_sh = mx > 0.f ? 1.0f / mx : 1.0f;
    }
    __syncthreads();
    const float sc = s_sh;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[i] * sc;
        const TL h = (TL)v;
        hi[i] = h;
        if (lo) lo[i] = (TL)(v - (float)h);
    }
}

template <typename TL>
__device__ inline floatx16 mfma32_lp(const typename LPVec<TL>::type &a, const typename LPVec<TL>::type &b, floatx16 c) {
    if constexpr (std::is_same<TL, __bf16>::value) return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// LDS position (16-byte units) of the 8-element group kq (0..3) of row r in a 32-element
// chunk row: 8 (and 16) consecutive rows read at one kq hit distinct bank groups.
__device__ inline int swz4(int r, int kq) { return r * 4 + (kq ^ (((r >> 1) ^ (r >> 3)) & 3)); }

__device__ inline void copy16_to_lds_b(const void *g, void *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0); }

// Six 16-byte LDS reads (byte addresses a[i]) completed before returning.
__device__ inline void lds_read6(const int *a, float4 *v) {
    asm volatile(
        "ds_read_b128 %0, %6\n"
        "ds_read_b128 %1, %7\n"
        "ds_read_b128 %2, %8\n"
        "ds_read_b128 %3, %9\n"
        "ds_read_b128 %4, %10\n"
        "ds_read_b128 %5, %11\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5])
        : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5])
        : "memory");
}

// Low-precision tap GEMM with both operands already split (A = A_hi + A_lo stored as
// operators, B = (B_hi + B_lo) * max|in| by split_lp_kernel): products on
// v_mfma_f32_32x32x16_{bf16,f16} with FP32 accumulation, NP = 1 (hi only) or 3
// (hi.hi + hi.lo + lo.hi).  BM = 128 rows x 64 boxes per workgroup, each wave 64 x 32;
// tiles are copied global -> LDS asynchronously three stages deep, as in tapgemm_f32.
template <typename TL, int NP, int NS, int PASS>
__global__ __launch_bounds__(256) void tapgemm_lp_staged(TapArgs<TL, TL, float> p) {
    static_assert(NS >= 3 && NS <= 6, "three to six stages");
    typedef typename LPVec<TL>::type vec8;
    constexpr int BM = 128, IM = 2, NPART = NP == 3 ? 2 : 1;
    constexpr int A_BYTES = BM * 64, B_BYTES = BN * 64;                 // one part of one tile
    constexpr int STG = NPART * (A_BYTES + B_BYTES);                      // bytes per stage
    constexpr int LPC = NPART * 3;                                        // copies per thread per chunk
    constexpr int NR = NPART * 6;                                         // fragment reads per chunk
    __shared__ __align__(16) char St[NS * STG];
    __shared__ float in_scale_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = p.groups;
    const int cls = blockIdx.z / G, grp = blockIdx.z % G;
    const int tpg = (p.ntaps + G - 1) / G;
    const int t0 = grp * tpg, t1 = min(p.ntaps, t0 + tpg);
    const int RT = (p.M + BM - 1) / BM;                 // row tiles: the fastest tile index
    const int64_t lin = p.in_nz || p.out_need ? sparse_tile(blockIdx.x, gridDim.x, RT)
                                              : xcd_tile(blockIdx.x, gridDim.x);
    const int64_t j0 = lin / RT * BN;
    const int m0 = (int)(lin % RT) * BM;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
    const int KC = p.K / 32;
    __shared__ uint8_t tap_flags[256];
    int act[4];
    const int nact = active_taps(p, cls, t0, t1, j0, tap_flags, act);   // taps with nonzero sources
    const int total = nact * KC;
    if (tid == 0) {
        float mx = 0.f;
        for (int i = 0; i < p.n_amax; ++i) mx = fmaxf(mx, p.amax[i]);
        in_scale_sh = mx > 0.f ? mx : 1.0f;
    }

    // NP = 3 folds the FP32 partial sums into FP64 totals every NS chunks; with NP = 1
    // the operand rounding (2^-9 or 2^-12) dwarfs FP32 accumulation and acc is the sum
    constexpr int NT = NP == 3 ? 16 : 1;
    floatx16 acc[IM];
    double tot[IM][NT];
#pragma unroll
    for (int i = 0; i < IM; ++i) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
#pragma unroll
        for (int v = 0; v < NT; ++v) tot[i][v] = 0.0;
    }
    int my_op[4], my_off[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = t0 + act[r];
        const bool live = 64 * r + lane < nact;
        my_op[r] = live ? tap_op_of(p.tap_op, p.inl_op, cls * p.ntaps + t) : 0;
        my_off[r] = live ? tap_op_of(p.tap_off, p.inl_off, cls * p.ntaps + t) : 0;
    }
    // copy r (0, 1) of this thread fills A position (r * 4 + wave) * 64 + lane; the B
    // position is wave * 64 + lane.  Positions are 16-byte groups.
    int a_off[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int pos = (r * 4 + wave) * 64 + lane, row = pos >> 2;
        const int kq = (pos & 3) ^ (((row >> 1) ^ (row >> 3)) & 3);
        a_off[r] = min(m0 + row, p.M - 1) * p.K + kq * 8;
    }
    const int bpos = wave * 64 + lane, bbox = bpos >> 2;
    const int b_kq = (bpos & 3) ^ (((bbox >> 1) ^ (bbox >> 3)) & 3);
    int64_t bsrc = -1;
    const TL *Ahi = p.A, *Alo = p.A2;
    auto issue = [&](int it, int stage) {
        const int tt = it / KC, kc = it % KC;
        if (kc == 0) {
            int op = 0, off = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if ((tt >> 6) == r) {
                    op = __builtin_amdgcn_readlane(my_op[r], tt & 63);
                    off = __builtin_amdgcn_readlane(my_off[r], tt & 63);
                }
            Ahi = p.A + (int64_t)op * p.a_stride;
            if (NP == 3) Alo = p.A2 + (int64_t)op * p.a_stride;
            const int64_t j = j0 + bbox;
            const int64_t src = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl, p.zroots) : -1;
            bsrc = src >= 0 ? src * p.in_ld + b_kq * 8 : -1;
        }
        const int k = kc * 32;
        char *S = St + stage * STG;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            copy16_to_lds_b(Ahi + a_off[r] + k, S + (r * 4 + wave) * 1024);
            if (NP == 3) copy16_to_lds_b(Alo + a_off[r] + k, S + A_BYTES + (r * 4 + wave) * 1024);
        }
        const TL *zero = (const TL *)kZeroChunk + b_kq * 8;
        copy16_to_lds_b(bsrc >= 0 ? p.in + bsrc + k : zero, S + NPART * A_BYTES + wave * 1024);
        if (NP == 3) copy16_to_lds_b(bsrc >= 0 ? p.in2 + bsrc + k : zero, S + NPART * A_BYTES + B_BYTES + wave * 1024);
    };

    // fragment addresses (stage 0): [A_hi (i, s)] [A_lo (i, s)] [B_hi s] [B_lo s], k group 2q + s
    const int q = lane >> 5, r32 = lane & 31;
    int fa[NR];
    {
        const int base = (int)(uintptr_t)(__attribute__((address_space(3))) char *)St;   // LDS byte address
        int n = 0;
        for (int part = 0; part < NPART; ++part)
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int s = 0; s < 2; ++s) fa[n++] = base + part * A_BYTES + swz4(wr + 32 * i + r32, 2 * q + s) * 16;
        for (int part = 0; part < NPART; ++part)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                fa[n++] = base + NPART * A_BYTES + part * B_BYTES + swz4(wc + r32, 2 * q + s) * 16;
    }
    auto as8 = [](const float4 &v) { vec8 r; __builtin_memcpy(&r, &v, 16); return r; };
    auto compute = [&](const float4 *fr, int it) {
        const float4 *Ah = fr, *Al = fr + 4, *Bh = fr + 4 * NPART, *Bl = fr + 4 * NPART + 2;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < IM; ++i) {
                acc[i] = mfma32_lp<TL>(as8(Ah[2 * i + s]), as8(Bh[s]), acc[i]);
                if (NP == 3) {
                    acc[i] = mfma32_lp<TL>(as8(Ah[2 * i + s]), as8(Bl[s]), acc[i]);
                    acc[i] = mfma32_lp<TL>(as8(Al[2 * i + s]), as8(Bh[s]), acc[i]);
                }
            }
    };
    auto fold = [&]() {   // FP64 totals take the FP32 partial sums of the last NS chunks
        if constexpr (NP == 3) {
#pragma unroll
            for (int i = 0; i < IM; ++i) {
#pragma unroll
                for (int v = 0; v < 16; ++v) { tot[i][v] += (double)acc[i][v]; acc[i][v] = 0.f; }
            }
        }
    };
    auto total_of = [&](int i, int v) -> double {
        if constexpr (NP == 3) return tot[i][v];
        else return (double)acc[i][v];
    };
    __syncthreads();   // in_scale_sh
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
        if (u < total) issue(u, u);
    float4 fr[NR];
    int it = 0;
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        const int c = it + u;
        if (c >= total) return false;
        // chunk c has landed for every wave; chunks c+1 .. c+NS-2 may still be in flight
        wait_outstanding_then_barrier<LPC>(min(total - 1 - c, NS - 2));
        int a[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) a[i] = fa[i] + u * STG;
        if constexpr (NR == 12) lds_read12(*(const int (*)[12])a, *(float4 (*)[12])fr);
        else lds_read6(a, fr);
        if (c + NS - 1 < total) issue(c + NS - 1, (u + NS - 1) % NS);
        compute(fr, c);
        return true;
    };
    for (; it < total; it += NS) {
        unrolled_steps(step, std::make_integer_sequence<int, NS>());
        fold();
    }
    const double oscale = (double)p.op_scale * (double)in_scale_sh;
    const int64_t j = j0 + wc + r32;
    if (j < p.n_per_class) {
        const int64_t b = (int64_t)p.cls_stride * j + cls;
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int row = m0 + wr + 32 * i + 8 * g + 4 * q;
                if (row < p.M) {
                    double v0 = total_of(i, 4 * g) * oscale, v1 = total_of(i, 4 * g + 1) * oscale;
                    double v2 = total_of(i, 4 * g + 2) * oscale, v3 = total_of(i, 4 * g + 3) * oscale;
                    float *o;
                    if (G > 1) {
                        o = p.part + ((int64_t)grp * p.n_boxes + b) * p.out_ld + row;
                    } else {
                        o = p.out + b * p.out_ld + row;
                        if (p.accumulate) {
                            const float4 old = *(const float4 *)o;
                            v0 += old.x; v1 += old.y; v2 += old.z; v3 += old.w;
                        }
                    }
                    *(float4 *)o = make_float4((float)v0, (float)v1, (float)v2, (float)v3);
                }
            }
    }
}

constexpr int64_t kTargetWGs = 2048;   // about 8 workgroups per CU
// The staged kernels hold two workgroups per CU; launches that split their taps do
// best with about one such wave of workgroups (measured on the 256^3 M2L levels).
constexpr int64_t kTargetWGsStaged = 512;
template <typename TA, typename TI, typename TO>
int choose_groups(const TapArgs<TA, TI, TO> &p, int bm, int64_t target) {
    if (!p.part || p.ntaps <= 1) return 1;
    const int64_t base = ((p.n_per_class + BN - 1) / BN) * ((p.M + bm - 1) / bm) * p.nclass;
    int64_t g = (target + base - 1) / base;
    if (g > p.ntaps) g = p.ntaps;
    // the scratch must hold g partial outputs
    while (g > 1 && g * p.n_boxes * p.out_ld > p.part_capacity) --g;
    if (g <= 1) return 1;
    // equal-size groups: no empty trailing group
    const int tpg = (p.ntaps + (int)g - 1) / (int)g;
    return (p.ntaps + tpg - 1) / tpg;
}

template <typename TA, typename TI, typename TO, typename F>
int launch_split(TapArgs<TA, TI, TO> p, int bm, F kernel, hipStream_t st, int64_t target = kTargetWGs) {
    p.groups = choose_groups(p, bm, target);
    dim3 grid((unsigned)(((p.n_per_class + BN - 1) / BN) * ((p.M + bm - 1) / bm)), 1u,
              (unsigned)(p.nclass * p.groups));
    hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    if (p.groups > 1) {
        const int64_t n = p.n_boxes * p.out_ld;
        int64_t blocks = (n + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(reduce_partials, dim3((unsigned)blocks), dim3(256), 0, st, (const float *)p.part,
                           p.groups, n, p.accumulate, (float *)p.out);
        KIFMM_HIP(hipGetLastError());
    }
    return KIFMM_OK;
}

}  // namespace

template <int PASS>
int run_f32_pass(const TapArgs<float, float, float> &p, hipStream_t st) {
    if (p.M > 64) return launch_split(p, 128, tapgemm_f32_staged<PASS>, st, kTargetWGsStaged);
    return launch_split(p, 64, tapgemm_f32_small<PASS>, st);
}

int run_tap_f32(const TapArgs<float, float, float> &p, hipStream_t st) {
    if (p.K % BK != 0) return fail(KIFMM_EINVAL, "tap GEMM: K not a multiple of 32");
    if (p.in_ld % 4 != 0) return fail(KIFMM_EINVAL, "tap GEMM: input stride not a multiple of 4");
    if (p.ntaps > 256) return fail(KIFMM_EINVAL, "tap GEMM: more than 256 taps");
    if (p.pass == PASS_P2P) return run_f32_pass<PASS_P2P>(p, st);
    if (p.pass == PASS_M2L) return run_f32_pass<PASS_M2L>(p, st);
    return run_f32_pass<PASS_GENERIC>(p, st);
}

int run_tap_f64(const TapArgs<double, double, double> &p0, hipStream_t st) {
    TapArgs<double, double, double> p = p0;
    p.groups = 1;
    dim3 grid((unsigned)((p.n_per_class + VN - 1) / VN), (unsigned)((p.M + VM - 1) / VM), p.nclass);
    hipLaunchKernelGGL(tapgemm_valu<double>, grid, dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename TL, bool X3, int PASS>
int run_lp_bm(const TapArgs<TL, float, float> &p, hipStream_t st) {
    if (p.M > 64) return launch_split(p, 128, tapgemm_lp<TL, X3, PASS, 128>, st);
    if (p.M > 32) return launch_split(p, 64, tapgemm_lp<TL, X3, PASS, 64>, st);
    return launch_split(p, 32, tapgemm_lp<TL, X3, PASS, 32>, st);
}

template <typename TL, bool X3>
int run_lp_pass(const TapArgs<TL, float, float> &p, hipStream_t st) {
    if (p.pass == PASS_P2P) return run_lp_bm<TL, X3, PASS_P2P>(p, st);
    if (p.pass == PASS_M2L) return run_lp_bm<TL, X3, PASS_M2L>(p, st);
    return run_lp_bm<TL, X3, PASS_GENERIC>(p, st);
}

template <typename TL>
int run_tap_lp(const TapArgs<TL, float, float> &p, bool x3, hipStream_t st) {
    if (p.K % LBK != 0) return fail(KIFMM_EINVAL, "tap GEMM (low precision): K not a multiple of 32");
    if (x3) {
        if constexpr (std::is_same<TL, __bf16>::value) return run_lp_pass<TL, true>(p, st);
        else return fail(KIFMM_EUNSUPPORTED, "split operands are implemented for bfloat16 only");
    }
    return run_lp_pass<TL, false>(p, st);
}
template int run_tap_lp<__bf16>(const TapArgs<__bf16, float, float> &, bool, hipStream_t);
template int run_tap_lp<_Float16>(const TapArgs<_Float16, float, float> &, bool, hipStream_t);

int run_wgrad(WgradArgs p, bool bf16, hipStream_t st) {
    if (p.M % 32 || p.K % 32) return fail(KIFMM_EINVAL, "weight gradient: channel counts must be multiples of 32");
    const int bw = (p.M % 64 == 0 && p.K % 64 == 0) ? 64 : 32;
    const int64_t tiles = (int64_t)(p.M / bw) * (p.K / bw);
    const int64_t wsize = (int64_t)p.ntaps * p.M * p.K;
    int64_t g = (kTargetWGs + tiles * p.ntaps - 1) / (tiles * p.ntaps);
    const int64_t gmax = (p.n_per_class + 255) / 256;          // at least 256 voxels per group
    if (g > gmax) g = gmax;
    if (!p.part) g = 1;
    while (g > 1 && g * wsize > p.part_capacity) --g;
    if (g < 1) g = 1;
    p.groups = (int)g;
    dim3 grid((unsigned)g, (unsigned)tiles, (unsigned)p.ntaps);
    if (bw == 64) {
        if (bf16) hipLaunchKernelGGL((wgrad_kernel<__bf16, 64>), grid, dim3(256), 0, st, p);
        else hipLaunchKernelGGL((wgrad_kernel<float, 64>), grid, dim3(256), 0, st, p);
    } else {
        if (bf16) hipLaunchKernelGGL((wgrad_kernel<__bf16, 32>), grid, dim3(256), 0, st, p);
        else hipLaunchKernelGGL((wgrad_kernel<float, 32>), grid, dim3(256), 0, st, p);
    }
    KIFMM_HIP(hipGetLastError());
    if (g > 1) {
        int64_t blocks = (wsize + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(reduce_partials, dim3((unsigned)blocks), dim3(256), 0, st, (const float *)p.part,
                           (int)g, wsize, 0, p.dw);
        KIFMM_HIP(hipGetLastError());
    }
    return KIFMM_OK;
}

int run_amax(const float *x, int64_t n, float *part, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(amax_partial, dim3(nparts), dim3(256), 0, st, x, n, part);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename TL>
int run_split_lp(const float *x, int64_t n, const float *amax, int n_amax, TL *hi, TL *lo, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(split_lp_kernel<TL>, dim3((unsigned)blocks), dim3(256), 0, st, x, n, amax, n_amax, hi, lo);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}
template int run_split_lp<__bf16>(const float *, int64_t, const float *, int, __bf16 *, __bf16 *, hipStream_t);
template int run_split_lp<_Float16>(const float *, int64_t, const float *, int, _Float16 *, _Float16 *, hipStream_t);

template <typename TL, int NP, int NS>
int run_staged_pass(const TapArgs<TL, TL, float> &p, hipStream_t st) {
    // single-part products are cheap enough that more, smaller tap groups pay
    const int64_t target = NP == 3 ? kTargetWGsStaged : kTargetWGs;
    if (p.pass == PASS_P2P) return launch_split(p, 128, tapgemm_lp_staged<TL, NP, NS, PASS_P2P>, st, target);
    if (p.pass == PASS_M2L) return launch_split(p, 128, tapgemm_lp_staged<TL, NP, NS, PASS_M2L>, st, target);
    return launch_split(p, 128, tapgemm_lp_staged<TL, NP, NS, PASS_GENERIC>, st, target);
}

template <typename TL>
int run_tap_lp_staged(const TapArgs<TL, TL, float> &p, bool x3, hipStream_t st) {
    if (p.K % 32 != 0) return fail(KIFMM_EINVAL, "tap GEMM (staged): K not a multiple of 32");
    if (p.in_ld % 8 != 0) return fail(KIFMM_EINVAL, "tap GEMM (staged): input stride not a multiple of 8");
    if (p.ntaps > 256) return fail(KIFMM_EINVAL, "tap GEMM (staged): more than 256 taps");
    if (x3) return run_staged_pass<TL, 3, 3>(p, st);
    return run_staged_pass<TL, 1, 3>(p, st);
}
template int run_tap_lp_staged<__bf16>(const TapArgs<__bf16, __bf16, float> &, bool, hipStream_t);
template int run_tap_lp_staged<_Float16>(const TapArgs<_Float16, _Float16, float> &, bool, hipStream_t);

}  // namespace kifmm
