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
// Kernels:
//   tapgemm_mfma_f32   FP32 on MFMA (v_mfma_f32_16x16x4f32), 64 x 64 output tile
//   tapgemm_mfma_lp    BF16 / FP16 operands (v_mfma_f32_16x16x32_{bf16,f16}),
//                      FP32 accumulate; the input vectors are scaled by a
//                      device-side factor and rounded to nearest-even on load
//   tapgemm_valu<T>    LDS-tiled VALU version for FP64 (and any T)
#include "common.h"
#include "tapgemm.h"

#include <type_traits>

namespace kifmm {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ inline int64_t source_box(int mode, int64_t b, int off, int nl) {
    switch (mode) {
        case SRC_SAME: return b;
        case SRC_CHILD: return 8 * b + off;
        case SRC_PARENT: return b >> 3;
        default: {
            int x, y, z;
            morton_decode((uint32_t)b, x, y, z);
            x += ((off >> 10) & 31) - 16;
            y += ((off >> 5) & 31) - 16;
            z += (off & 31) - 16;
            if (x < 0 || y < 0 || z < 0 || x >= nl || y >= nl || z >= nl) return -1;
            return (int64_t)morton_encode(x, y, z);
        }
    }
}

constexpr int BM = 64, BN = 64, BK = 16, PADK = 4;
constexpr int kFoldK = 32;

__global__ __launch_bounds__(256) void tapgemm_mfma_f32(TapArgs<float, float, float> p) {
    __shared__ float As[BM][BK + PADK];
    __shared__ float Bs[BN][BK + PADK];
    __shared__ int64_t srcs[BN];
    const int cls = blockIdx.z;
    const int64_t j0 = (int64_t)blockIdx.x * BN;
    const int m0 = blockIdx.y * BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // MFMA partial sums run over at most kFoldK reduction elements (kFoldK / 4
    // chained FP32 steps) before they are added into FP64 totals, which keeps
    // the rounding of long near-field and M2L sums at the level of one short chain.
    floatx4 acc[2][2];
    double tot[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[i][j][v] = 0.0;
        }
    auto fold = [&]() {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
                for (int v = 0; v < 4; ++v) tot[i][j][v] += (double)acc[i][j][v];
                acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    };

    const int lr = tid >> 2, lk = (tid & 3) * 4;  // loader coordinates
    for (int t = 0; t < p.ntaps; ++t) {
        const int op = p.tap_op[cls * p.ntaps + t];
        const int off = p.tap_off[cls * p.ntaps + t];
        __syncthreads();  // all readers of the previous tap's srcs are done
        int64_t s = -1;
        if (tid < BN) {
            const int64_t j = j0 + tid;
            if (j < p.n_per_class) s = source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl);
            srcs[tid] = s;
        }
        if (!__syncthreads_or(s >= 0)) continue;
        const float *Aop = p.A + (int64_t)op * p.a_stride;
        const int64_t mysrc = srcs[lr];
        for (int k0 = 0; k0 < p.K; k0 += BK) {
            float4 av = make_float4(0.f, 0.f, 0.f, 0.f), bv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (m0 + lr < p.M) av = *(const float4 *)(Aop + (int64_t)(m0 + lr) * p.K + k0 + lk);
            if (mysrc >= 0) bv = *(const float4 *)(p.in + mysrc * p.in_ld + k0 + lk);
            __syncthreads();
            *(float4 *)&As[lr][lk] = av;
            *(float4 *)&Bs[lr][lk] = bv;
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kl = kk + (lane >> 4);
                float a0 = As[wr + (lane & 15)][kl], a1 = As[wr + 16 + (lane & 15)][kl];
                float b0 = Bs[wc + (lane & 15)][kl], b1 = Bs[wc + 16 + (lane & 15)][kl];
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
            if (((k0 + BK) % kFoldK) == 0 || k0 + BK >= p.K) fold();
        }
    }
    // D layout of 16x16x4: lane holds rows 4*(lane/16)+v, column lane%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int row = m0 + wr + 16 * i + 4 * (lane >> 4);
            const int64_t j = j0 + wc + 16 * jj + (lane & 15);
            if (row < p.M && j < p.n_per_class) {
                const int64_t b = (int64_t)p.cls_stride * j + cls;
                float *o = p.out + b * p.out_ld + row;
                double v0 = tot[i][jj][0], v1 = tot[i][jj][1], v2 = tot[i][jj][2], v3 = tot[i][jj][3];
                if (p.accumulate) {
                    const float4 old = *(const float4 *)o;
                    v0 += old.x; v1 += old.y; v2 += old.z; v3 += old.w;
                }
                *(float4 *)o = make_float4((float)v0, (float)v1, (float)v2, (float)v3);
            }
        }
}

// Low-precision operands: A pre-rounded to TL, input FP32 scaled and rounded on load.
template <typename TL>
struct LPVec;
template <> struct LPVec<__bf16> { typedef bf16x8 type; };
template <> struct LPVec<_Float16> { typedef halfx8 type; };

constexpr int LBK = 32, LPAD = 8;

template <typename TL>
__global__ __launch_bounds__(256) void tapgemm_mfma_lp(TapArgs<TL, float, float> p) {
    typedef typename LPVec<TL>::type vec8;
    __shared__ TL As[BM][LBK + LPAD];
    __shared__ TL Bs[BN][LBK + LPAD];
    __shared__ int64_t srcs[BN];
    __shared__ float in_scale_sh;
    const int cls = blockIdx.z;
    const int64_t j0 = (int64_t)blockIdx.x * BN;
    const int m0 = blockIdx.y * BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // input scale = 1 / max|in|, from per-block partial maxima
    if (tid == 0) {
        float mx = 0.f;
        for (int i = 0; i < p.n_amax; ++i) mx = fmaxf(mx, p.amax[i]);
        in_scale_sh = mx > 0.f ? 1.0f / mx : 1.0f;
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    const float sin = in_scale_sh;
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    for (int t = 0; t < p.ntaps; ++t) {
        const int op = p.tap_op[cls * p.ntaps + t];
        const int off = p.tap_off[cls * p.ntaps + t];
        __syncthreads();  // all readers of the previous tap's srcs are done
        int64_t s = -1;
        if (tid < BN) {
            const int64_t j = j0 + tid;
            if (j < p.n_per_class) s = source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl);
            srcs[tid] = s;
        }
        if (!__syncthreads_or(s >= 0)) continue;
        const TL *Aop = p.A + (int64_t)op * p.a_stride;
        const int64_t mysrc = srcs[lr];
        for (int k0 = 0; k0 < p.K; k0 += LBK) {
            vec8 av, bv;
            if (m0 + lr < p.M) av = *(const vec8 *)(Aop + (int64_t)(m0 + lr) * p.K + k0 + lk);
            else for (int e = 0; e < 8; ++e) av[e] = (TL)0.f;
            if (mysrc >= 0) {
                const float4 x0 = *(const float4 *)(p.in + mysrc * p.in_ld + k0 + lk);
                const float4 x1 = *(const float4 *)(p.in + mysrc * p.in_ld + k0 + lk + 4);
                bv[0] = (TL)(x0.x * sin); bv[1] = (TL)(x0.y * sin);
                bv[2] = (TL)(x0.z * sin); bv[3] = (TL)(x0.w * sin);
                bv[4] = (TL)(x1.x * sin); bv[5] = (TL)(x1.y * sin);
                bv[6] = (TL)(x1.z * sin); bv[7] = (TL)(x1.w * sin);
            } else {
                for (int e = 0; e < 8; ++e) bv[e] = (TL)0.f;
            }
            __syncthreads();
            *(vec8 *)&As[lr][lk] = av;
            *(vec8 *)&Bs[lr][lk] = bv;
            __syncthreads();
            const int kl = 8 * (lane >> 4);
            const vec8 a0 = *(const vec8 *)&As[wr + (lane & 15)][kl];
            const vec8 a1 = *(const vec8 *)&As[wr + 16 + (lane & 15)][kl];
            const vec8 b0 = *(const vec8 *)&Bs[wc + (lane & 15)][kl];
            const vec8 b1 = *(const vec8 *)&Bs[wc + 16 + (lane & 15)][kl];
            if constexpr (std::is_same<TL, __bf16>::value) {
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
            } else {
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
    }
    const float oscale = p.op_scale / sin;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int row = m0 + wr + 16 * i + 4 * (lane >> 4);
            const int64_t j = j0 + wc + 16 * jj + (lane & 15);
            if (row < p.M && j < p.n_per_class) {
                const int64_t b = (int64_t)p.cls_stride * j + cls;
                float *o = p.out + b * p.out_ld + row;
                floatx4 v = acc[i][jj];
                v[0] *= oscale; v[1] *= oscale; v[2] *= oscale; v[3] *= oscale;
                if (p.accumulate) {
                    const float4 old = *(const float4 *)o;
                    v[0] += old.x; v[1] += old.y; v[2] += old.z; v[3] += old.w;
                }
                *(float4 *)o = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
}

// Generic LDS-tiled VALU version: 64 rows x 32 boxes per workgroup, each thread
// 4 rows x 2 boxes.
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
        const int op = p.tap_op[cls * p.ntaps + t];
        const int off = p.tap_off[cls * p.ntaps + t];
        __syncthreads();
        if (tid < VN) {
            const int64_t j = j0 + tid;
            srcs[tid] = j < p.n_per_class ? source_box(p.mode, (int64_t)p.cls_stride * j + cls, off, p.nl) : -1;
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

template <typename TA, typename TI, typename TO>
dim3 grid_of(const TapArgs<TA, TI, TO> &p, int bn, int bm) {
    return dim3((unsigned)((p.n_per_class + bn - 1) / bn), (unsigned)((p.M + bm - 1) / bm), p.nclass);
}

}  // namespace

int run_tap_f32(const TapArgs<float, float, float> &p, hipStream_t st) {
    if (p.K % BK != 0) return fail(KIFMM_EINVAL, "tap GEMM: K not a multiple of 16");
    hipLaunchKernelGGL(tapgemm_mfma_f32, grid_of(p, BN, BM), dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_tap_f64(const TapArgs<double, double, double> &p, hipStream_t st) {
    hipLaunchKernelGGL(tapgemm_valu<double>, grid_of(p, VN, VM), dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int run_tap_f32_valu(const TapArgs<float, float, float> &p, hipStream_t st) {
    hipLaunchKernelGGL(tapgemm_valu<float>, grid_of(p, VN, VM), dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

template <typename TL>
int run_tap_lp(const TapArgs<TL, float, float> &p, hipStream_t st) {
    if (p.K % LBK != 0) return fail(KIFMM_EINVAL, "tap GEMM (low precision): K not a multiple of 32");
    hipLaunchKernelGGL(tapgemm_mfma_lp<TL>, grid_of(p, BN, BM), dim3(256), 0, st, p);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}
template int run_tap_lp<__bf16>(const TapArgs<__bf16, float, float> &, hipStream_t);
template int run_tap_lp<_Float16>(const TapArgs<_Float16, float, float> &, hipStream_t);

int run_amax(const float *x, int64_t n, float *part, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(amax_partial, dim3(nparts), dim3(256), 0, st, x, n, part);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // namespace kifmm
