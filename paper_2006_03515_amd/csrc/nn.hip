// Kernels of the learned surrogate: a 3D convolutional encoder-decoder mapping a
// coarse source field to S_ph (not in the paper; it approximates the map of
// eq. (integral) and is judged by the FMM).
//
// Activations are FP32, channels-last, voxels in Morton order per sample:
// x[(s * n^3 + morton(i, j, k)) * C + c].  In that order every layer is a tap GEMM
// of csrc/tapgemm.hip:
//   CONV3  3x3x3, stride 1, zero padding: 27 neighbour taps (SRC_NBR)
//   DOWN2  2x2x2, stride 2: the 8 children of a coarse voxel are consecutive (SRC_CHILD)
//   UP2    transposed 2x2x2, stride 2: fine voxel 8J + c reads coarse J with W_c (SRC_PARENT)
//   POINT  1x1x1 (SRC_SAME)
// and the data gradient of each is the tap GEMM of the adjoint mode with transposed
// weights (CONV3 with negated offsets, DOWN2 <-> UP2).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.h"
#include "tapgemm.h"

namespace kifmm {

namespace {

constexpr int kT = 256;

unsigned blocks(int64_t n, int64_t cap = 65536) {
    int64_t b = (n + kT - 1) / kT;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

// w [taps][co][ci] FP32 -> forward copy [taps][co][ci] and transposed [taps][ci][co] (T)
template <typename T>
__global__ void prepare_weights_kernel(int taps, int co, int ci, const float *__restrict__ w,
                                       T *__restrict__ wf, T *__restrict__ wb) {
    const int64_t n = (int64_t)taps * co * ci;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e / ((int64_t)co * ci));
        const int r = (int)((e / ci) % co), c = (int)(e % ci);
        const T v = (T)w[e];
        if (wf) wf[e] = v;
        if (wb) wb[((int64_t)t * ci + c) * co + r] = v;
    }
}

// y = act(y + bias), act = leaky ReLU with slope alpha (alpha = 1: identity)
__global__ void bias_act_kernel(int64_t nvox, int c, float *__restrict__ y, const float *__restrict__ bias,
                                float alpha) {
    const int64_t n = nvox * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        float v = y[e] + (bias ? bias[e % c] : 0.f);
        y[e] = v > 0.f ? v : alpha * v;
    }
}

// dy <- dy * act'(pre) using the post-activation sign (alpha > 0); per-block
// per-channel partial sums of the result for the bias gradient
__global__ void bias_act_bwd_kernel(int64_t nvox, int c, const float *__restrict__ y, float *__restrict__ dy,
                                    float alpha, int64_t vox_per_block, float *__restrict__ part) {
    // one block handles voxels [b*vpb, (b+1)*vpb); thread layout: channel = tid % c
    const int64_t v0 = blockIdx.x * vox_per_block;
    const int64_t v1 = min(nvox, v0 + vox_per_block);
    const int ch = threadIdx.x % c, lanes = blockDim.x / c, li = threadIdx.x / c;
    double s = 0.0;
    if (li < lanes) {
        for (int64_t v = v0 + li; v < v1; v += lanes) {
            const int64_t e = v * c + ch;
            const float g = y[e] > 0.f ? dy[e] : alpha * dy[e];
            dy[e] = g;
            s += g;
        }
    }
    __shared__ double sh[kT];
    sh[threadIdx.x] = (li < lanes) ? s : 0.0;
    __syncthreads();
    if (threadIdx.x < c) {
        double tsum = 0.0;
        for (int l = 0; l < lanes; ++l) tsum += sh[l * c + threadIdx.x];
        part[(int64_t)blockIdx.x * c + threadIdx.x] = (float)tsum;
    }
}

__global__ void sum_rows_kernel(const float *__restrict__ part, int nrows, int c, float *__restrict__ out) {
    const int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= c) return;
    double s = 0.0;
    for (int r = 0; r < nrows; ++r) s += part[(int64_t)r * c + ch];
    out[ch] = (float)s;
}

__device__ inline double block_sum_d(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    return r;
}

// prediction y[(s*V + morton(g)) * ld] (channel 0) vs target t[s*V + g] (grid order):
// partial sums of (y - t)^2 and t^2 per (sample, block)
__global__ void loss_partial_kernel(int n, int64_t V, const float *__restrict__ y, int ld,
                                    const float *__restrict__ t, int nblk, double *__restrict__ part) {
    __shared__ double sh[4];
    const int s = blockIdx.y, b = blockIdx.x;
    double a = 0.0, c = 0.0;
    for (int64_t g = (int64_t)b * blockDim.x + threadIdx.x; g < V; g += (int64_t)nblk * blockDim.x) {
        const int i = (int)(g / ((int64_t)n * n)), j = (int)((g / n) % n), k = (int)(g % n);
        const int64_t m = morton_encode(i, j, k);
        const double yv = y[((int64_t)s * V + m) * ld], tv = t[(int64_t)s * V + g];
        a += (yv - tv) * (yv - tv);
        c += tv * tv;
    }
    a = block_sum_d(a, sh);
    c = block_sum_d(c, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)s * nblk + b) * 2] = a;
        part[((int64_t)s * nblk + b) * 2 + 1] = c;
    }
}

// per sample: loss_s = sum_a / sum_c; total = mean over samples
__global__ void loss_final_kernel(int batch, int nblk, const double *__restrict__ part, double *__restrict__ loss,
                                  double *__restrict__ tnorm) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double tot = 0.0;
    for (int s = 0; s < batch; ++s) {
        double a = 0.0, c = 0.0;
        for (int b = 0; b < nblk; ++b) {
            a += part[((int64_t)s * nblk + b) * 2];
            c += part[((int64_t)s * nblk + b) * 2 + 1];
        }
        tnorm[s] = c;
        loss[1 + s] = a / c;
        tot += a / c;
    }
    loss[0] = tot / batch;
}

// dy (same layout as y, channel 0, other channels zero) = 2 (y - t) / (||t||^2 batch)
__global__ void loss_grad_kernel(int n, int64_t V, int batch, const float *__restrict__ y, int ld,
                                 const float *__restrict__ t, const double *__restrict__ tnorm,
                                 float *__restrict__ dy) {
    const int64_t total = (int64_t)batch * V;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / V);
        const int64_t g = e % V;
        const int i = (int)(g / ((int64_t)n * n)), j = (int)((g / n) % n), k = (int)(g % n);
        const int64_t m = morton_encode(i, j, k);
        const int64_t o = ((int64_t)s * V + m) * ld;
        dy[o] = (float)(2.0 * ((double)y[o] - (double)t[e]) / (tnorm[s] * batch));
        for (int c = 1; c < ld; ++c) dy[o + c] = 0.f;
    }
}

__global__ void adam_kernel(int64_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// 27-neighbourhood features of the scaled field: feat[(s*V + morton(i,j,k)) * 32 + c],
// c = (dz+1)*9 + (dy+1)*3 + (dx+1) < 27 takes grid[s][i+dz][j+dy][k+dx] (0 outside); 27..31 are 0
__global__ void pack_input_kernel(int batch, int n, const float *__restrict__ grid, const float *__restrict__ scale,
                                  float *__restrict__ feat) {
    const int64_t V = (int64_t)n * n * n, total = (int64_t)batch * V;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / V);
        const int64_t g = e % V;
        const int i = (int)(g / ((int64_t)n * n)), j = (int)((g / n) % n), k = (int)(g % n);
        const float sc = scale ? scale[s] : 1.f;
        float *o = feat + ((int64_t)s * V + morton_encode(i, j, k)) * 32;
        int c = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx, ++c) {
                    const int a = i + dz, b = j + dy, d = k + dx;
                    o[c] = (a >= 0 && a < n && b >= 0 && b < n && d >= 0 && d < n)
                               ? grid[(int64_t)s * V + ((int64_t)a * n + b) * n + d] * sc
                               : 0.f;
                }
        for (; c < 32; ++c) o[c] = 0.f;
    }
}

// grid[s][g] = y[(s*V + morton(g)) * ld] * scale[s]
__global__ void unpack_output_kernel(int batch, int n, const float *__restrict__ y, int ld,
                                     const float *__restrict__ scale, float *__restrict__ grid) {
    const int64_t V = (int64_t)n * n * n, total = (int64_t)batch * V;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / V);
        const int64_t g = e % V;
        const int i = (int)(g / ((int64_t)n * n)), j = (int)((g / n) % n), k = (int)(g % n);
        grid[e] = y[((int64_t)s * V + morton_encode(i, j, k)) * ld] * (scale ? scale[s] : 1.f);
    }
}

// per (sample, block) partial max |x|
__global__ void max_abs_partial_kernel(int64_t V, const float *__restrict__ x, int nblk, float *__restrict__ part) {
    __shared__ float sh[4];
    const int s = blockIdx.y;
    float m = 0.f;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < V; g += (int64_t)nblk * blockDim.x)
        m = fmaxf(m, fabsf(x[(int64_t)s * V + g]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)s * nblk + blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// out[s] = 1 / max|x_s| (1 if the field is zero)
__global__ void max_abs_final_kernel(int batch, int nblk, const float *__restrict__ part, float *__restrict__ out,
                                     int reciprocal) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    float m = 0.f;
    for (int b = 0; b < nblk; ++b) m = fmaxf(m, part[(int64_t)s * nblk + b]);
    out[s] = reciprocal ? (m > 0.f ? 1.f / m : 1.f) : m;
}

// 2x2x2 block means, grid order: coarse[s][I][J][K] = mean of fine[s][2I+a][2J+b][2K+c]
__global__ void coarsen2_kernel(int batch, int nc, const float *__restrict__ fine, float *__restrict__ coarse) {
    const int nf = 2 * nc;
    const int64_t Vc = (int64_t)nc * nc * nc, Vf = (int64_t)nf * nf * nf, total = (int64_t)batch * Vc;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / Vc);
        const int64_t g = e % Vc;
        const int I = (int)(g / ((int64_t)nc * nc)), J = (int)((g / nc) % nc), Kk = (int)(g % nc);
        float acc = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    acc += fine[(int64_t)s * Vf + ((int64_t)(2 * I + a) * nf + (2 * J + b)) * nf + (2 * Kk + c)];
        coarse[e] = acc * 0.125f;
    }
}

// trilinear interpolation from the coarse cell centres to the fine cell centres;
// fine centre i sits at coarse coordinate (i + 0.5)/2 - 0.5, clamped to [0, nc-1]
__device__ inline void tri_axis(int i, int nc, int &i0, int &i1, float &w1) {
    float x = (i + 0.5f) * 0.5f - 0.5f;
    if (x < 0.f) x = 0.f;
    if (x > nc - 1.f) x = nc - 1.f;
    i0 = (int)floorf(x);
    i1 = min(i0 + 1, nc - 1);
    w1 = x - i0;
}

__global__ void upsample2_kernel(int batch, int nc, const float *__restrict__ coarse, float *__restrict__ fine) {
    const int nf = 2 * nc;
    const int64_t Vc = (int64_t)nc * nc * nc, Vf = (int64_t)nf * nf * nf, total = (int64_t)batch * Vf;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / Vf);
        const int64_t g = e % Vf;
        const int i = (int)(g / ((int64_t)nf * nf)), j = (int)((g / nf) % nf), k = (int)(g % nf);
        int a0, a1, b0, b1, c0, c1;
        float wa, wb, wc;
        tri_axis(i, nc, a0, a1, wa);
        tri_axis(j, nc, b0, b1, wb);
        tri_axis(k, nc, c0, c1, wc);
        const float *C = coarse + (int64_t)s * Vc;
        auto at = [&](int a, int b, int c) { return C[((int64_t)a * nc + b) * nc + c]; };
        const float v = (1 - wa) * ((1 - wb) * ((1 - wc) * at(a0, b0, c0) + wc * at(a0, b0, c1)) +
                                    wb * ((1 - wc) * at(a0, b1, c0) + wc * at(a0, b1, c1))) +
                        wa * ((1 - wb) * ((1 - wc) * at(a1, b0, c0) + wc * at(a1, b0, c1)) +
                              wb * ((1 - wc) * at(a1, b1, c0) + wc * at(a1, b1, c1)));
        fine[e] = v;
    }
}

// out = ||S[tgt] * scale - ref|| / ||ref||, one block, fixed-order reduction
__global__ void sampled_err_kernel(int64_t nt, const float *__restrict__ S, const int64_t *__restrict__ tgt,
                                   const double *__restrict__ ref, double scale, double *__restrict__ out) {
    __shared__ double sh[4];
    double a = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < nt; i += blockDim.x) {
        const double d = (double)S[tgt[i]] * scale - ref[i];
        a += d * d;
        c += ref[i] * ref[i];
    }
    a = block_sum_d(a, sh);
    c = block_sum_d(c, sh);
    if (threadIdx.x == 0) out[0] = c > 0 ? sqrt(a / c) : 0.0;
}

// x *= s
__global__ void scale_kernel(int64_t n, float *__restrict__ x, float s) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= s;
}

__global__ void add_kernel(int64_t n, const float *__restrict__ x, float *__restrict__ y) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] += x[e];
}

// out[0] = ||S[tgt] - R[tgt]|| / ||R[tgt]|| (two FP32 fields compared at the targets)
__global__ void sampled_diff_kernel(int64_t nt, const float *__restrict__ S, const float *__restrict__ R,
                                    const int64_t *__restrict__ tgt, double *__restrict__ out) {
    __shared__ double sh[4];
    double a = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < nt; i += blockDim.x) {
        const double r = (double)R[tgt[i]];
        const double d = (double)S[tgt[i]] - r;
        a += d * d;
        c += r * r;
    }
    a = block_sum_d(a, sh);
    c = block_sum_d(c, sh);
    if (threadIdx.x == 0) out[0] = c > 0 ? sqrt(a / c) : 0.0;
}

int pack(int x, int y, int z) { return ((x + 16) << 10) | ((y + 16) << 5) | (z + 16); }

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_kind(int kind, int n_in) {
    if (kind < KIFMM_NN_CONV3 || kind > KIFMM_NN_POINT) return fail(KIFMM_EINVAL, "unknown layer kind");
    if (!pow2(n_in) || n_in > 1024) return fail(KIFMM_EINVAL, "grid side must be a power of two <= 1024");
    if (kind == KIFMM_NN_DOWN2 && n_in < 2) return fail(KIFMM_EINVAL, "DOWN2 needs n_in >= 2");
    return KIFMM_OK;
}

int taps_of(int kind) { return kind == KIFMM_NN_CONV3 ? 27 : (kind == KIFMM_NN_POINT ? 1 : 8); }

// Fill the tap table of a forward (adjoint = false) or data-gradient (adjoint = true) launch.
template <typename TA>
void set_taps(TapArgs<TA, float, float> &p, int kind, bool adjoint, int batch, int n_in) {
    const int64_t nb = batch;
    int mode, nclass = 1, stride = 1, ntaps = 1, nl = 0;
    int64_t nper;
    const int n_out = kind == KIFMM_NN_DOWN2 ? n_in / 2 : (kind == KIFMM_NN_UP2 ? 2 * n_in : n_in);
    // the "output" of the launch: forward -> layer output, adjoint -> layer input
    const int n_launch_out = adjoint ? n_in : n_out;
    const int64_t Vout = (int64_t)n_launch_out * n_launch_out * n_launch_out;
    if (kind == KIFMM_NN_CONV3) {
        mode = SRC_NBR; ntaps = 27; nl = n_in; nper = nb * Vout;
        int t = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx, ++t) {
                    p.inl_op[t] = t;
                    p.inl_off[t] = adjoint ? pack(-dz, -dy, -dx) : pack(dz, dy, dx);
                }
    } else if (kind == KIFMM_NN_POINT) {
        mode = SRC_SAME; nper = nb * Vout;
        p.inl_op[0] = 0; p.inl_off[0] = 0;
    } else {
        const bool child = (kind == KIFMM_NN_DOWN2) != adjoint;   // DOWN2 fwd, UP2 adjoint
        if (child) {
            mode = SRC_CHILD; ntaps = 8; nper = nb * Vout;
            for (int c = 0; c < 8; ++c) { p.inl_op[c] = c; p.inl_off[c] = c; }
        } else {
            mode = SRC_PARENT; nclass = 8; stride = 8; nper = nb * Vout / 8;
            for (int c = 0; c < 8; ++c) { p.inl_op[c] = c; p.inl_off[c] = 0; }
        }
    }
    p.mode = mode; p.nl = nl; p.nclass = nclass; p.cls_stride = stride; p.n_per_class = nper;
    p.n_boxes = nper * nclass; p.ntaps = ntaps; p.tap_op = nullptr; p.tap_off = nullptr;
}

template <typename TA>
int run_layer(int kind, bool adjoint, int batch, int n_in, const float *x, int kin, const void *w, int mout,
              float *y, int accumulate, float *work, int64_t work_floats, hipStream_t st) {
    TapArgs<TA, float, float> p{};
    p.A = (const TA *)w; p.A2 = nullptr;
    p.a_stride = (int64_t)mout * kin; p.M = mout; p.K = kin;
    p.in = x; p.in_ld = kin; p.out = y; p.out_ld = mout;
    p.accumulate = accumulate;
    p.part = work; p.part_capacity = work ? work_floats : 0; p.groups = 1;
    p.amax = nullptr; p.n_amax = 0; p.op_scale = 1.0f; p.pass = PASS_GENERIC;
    set_taps(p, kind, adjoint, batch, n_in);
    if constexpr (std::is_same<TA, float>::value) return run_tap_f32(p, st);
    else return run_tap_lp<__bf16>(p, false, st);
}

int layer_checks(int kind, int batch, int n_in, const void *a, const void *b, const void *c, int kin, int mout) {
    KIFMM_TRY_(check_kind(kind, n_in));
    if (batch < 1) return fail(KIFMM_EINVAL, "batch must be >= 1");
    if (!a || !b || !c) return fail(KIFMM_EINVAL, "null pointer");
    if (kin <= 0 || kin % 32) return fail(KIFMM_EINVAL, "reduction channel count must be a positive multiple of 32");
    if (mout <= 0 || mout % 16) return fail(KIFMM_EINVAL, "output channel count must be a positive multiple of 16");
    return KIFMM_OK;
}

}  // namespace
}  // namespace kifmm

using namespace kifmm;

extern "C" {

int kifmm_nn_layer_forward(int32_t kind, int32_t batch, int32_t n_in, const float *x, int32_t ci, const void *w,
                           int32_t co, float *y, int32_t accumulate, int32_t bf16, float *work,
                           int64_t work_floats, void *stream) {
    KIFMM_TRY_(layer_checks(kind, batch, n_in, x, w, y, ci, co));
    if (bf16) return run_layer<__bf16>(kind, false, batch, n_in, x, ci, w, co, y, accumulate, work, work_floats,
                                       (hipStream_t)stream);
    return run_layer<float>(kind, false, batch, n_in, x, ci, w, co, y, accumulate, work, work_floats,
                            (hipStream_t)stream);
}

int kifmm_nn_layer_backward_data(int32_t kind, int32_t batch, int32_t n_in, const float *dy, int32_t co,
                                 const void *wt, int32_t ci, float *dx, int32_t accumulate, int32_t bf16,
                                 float *work, int64_t work_floats, void *stream) {
    KIFMM_TRY_(layer_checks(kind, batch, n_in, dy, wt, dx, co, ci));
    if (bf16) return run_layer<__bf16>(kind, true, batch, n_in, dy, co, wt, ci, dx, accumulate, work, work_floats,
                                       (hipStream_t)stream);
    return run_layer<float>(kind, true, batch, n_in, dy, co, wt, ci, dx, accumulate, work, work_floats,
                            (hipStream_t)stream);
}

int kifmm_nn_layer_backward_weight(int32_t kind, int32_t batch, int32_t n_in, const float *x, int32_t ci,
                                   const float *dy, int32_t co, float *dw, int32_t bf16, float *work,
                                   int64_t work_floats, void *stream) {
    KIFMM_TRY_(check_kind(kind, n_in));
    if (batch < 1 || !x || !dy || !dw) return fail(KIFMM_EINVAL, "null pointer or batch < 1");
    if (ci % 32 || co % 32 || ci <= 0 || co <= 0)
        return fail(KIFMM_EINVAL, "weight gradient: channel counts must be positive multiples of 32");
    WgradArgs p{};
    p.dy = dy; p.x = x; p.dw = dw; p.M = co; p.K = ci;
    p.part = work; p.part_capacity = work ? work_floats : 0;
    const int n_out = kind == KIFMM_NN_DOWN2 ? n_in / 2 : (kind == KIFMM_NN_UP2 ? 2 * n_in : n_in);
    const int64_t Vin = (int64_t)n_in * n_in * n_in, Vout = (int64_t)n_out * n_out * n_out;
    p.ntaps = taps_of(kind);
    if (kind == KIFMM_NN_CONV3) {
        p.mode = SRC_NBR; p.nl = n_in; p.cls_stride = 1; p.class_is_tap = 0; p.n_per_class = (int64_t)batch * Vout;
        int t = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dyy = -1; dyy <= 1; ++dyy)
                for (int dx = -1; dx <= 1; ++dx, ++t) p.tap_off[t] = pack(dz, dyy, dx);
    } else if (kind == KIFMM_NN_POINT) {
        p.mode = SRC_SAME; p.cls_stride = 1; p.class_is_tap = 0; p.n_per_class = (int64_t)batch * Vout;
        p.tap_off[0] = 0;
    } else if (kind == KIFMM_NN_DOWN2) {
        p.mode = SRC_CHILD; p.cls_stride = 1; p.class_is_tap = 0; p.n_per_class = (int64_t)batch * Vout;
        for (int c = 0; c < 8; ++c) p.tap_off[c] = c;
    } else {
        p.mode = SRC_PARENT; p.cls_stride = 8; p.class_is_tap = 1; p.n_per_class = (int64_t)batch * Vin;
        for (int c = 0; c < 8; ++c) p.tap_off[c] = 0;
    }
    return run_wgrad(p, bf16 != 0, (hipStream_t)stream);
}

int kifmm_nn_prepare_weights(int32_t taps, int32_t co, int32_t ci, const float *w, void *w_fwd, void *w_bwd,
                             int32_t bf16, void *stream) {
    if (taps <= 0 || co <= 0 || ci <= 0 || !w) return fail(KIFMM_EINVAL, "bad weight shape or null pointer");
    const int64_t n = (int64_t)taps * co * ci;
    if (bf16)
        hipLaunchKernelGGL(prepare_weights_kernel<__bf16>, dim3(blocks(n)), dim3(kT), 0, (hipStream_t)stream, taps,
                           co, ci, w, (__bf16 *)w_fwd, (__bf16 *)w_bwd);
    else
        hipLaunchKernelGGL(prepare_weights_kernel<float>, dim3(blocks(n)), dim3(kT), 0, (hipStream_t)stream, taps,
                           co, ci, w, (float *)w_fwd, (float *)w_bwd);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_bias_act(int64_t nvox, int32_t c, float *y, const float *bias, float alpha, void *stream) {
    if (nvox < 0 || c <= 0 || !y) return fail(KIFMM_EINVAL, "bad size or null pointer");
    hipLaunchKernelGGL(bias_act_kernel, dim3(blocks(nvox * c)), dim3(kT), 0, (hipStream_t)stream, nvox, c, y, bias,
                       alpha);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_bias_act_backward(int64_t nvox, int32_t c, const float *y, float *dy, float *dbias, float alpha,
                               float *work, int64_t work_floats, void *stream) {
    if (nvox <= 0 || c <= 0 || c > kT || !y || !dy) return fail(KIFMM_EINVAL, "bad size (1 <= c <= 256) or null");
    int64_t nblk = std::min<int64_t>(1024, (nvox + 255) / 256);
    if (dbias) {
        if (!work) return fail(KIFMM_EINVAL, "bias gradient needs work space");
        nblk = std::min<int64_t>(nblk, work_floats / c);
        if (nblk < 1) return fail(KIFMM_EINVAL, "work space too small");
    }
    const int64_t vpb = (nvox + nblk - 1) / nblk;
    float *part = dbias ? work : nullptr;
    if (!part) {
        // no bias: still apply the activation derivative; partial sums go to a dummy row
        return fail(KIFMM_EINVAL, "dbias must be non-NULL");
    }
    hipLaunchKernelGGL(bias_act_bwd_kernel, dim3((unsigned)nblk), dim3(kT), 0, (hipStream_t)stream, nvox, c, y, dy,
                       alpha, vpb, part);
    KIFMM_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_rows_kernel, dim3((c + 63) / 64), dim3(64), 0, (hipStream_t)stream, part, (int)nblk, c,
                       dbias);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_rel_l2_loss(int32_t batch, int32_t n, const float *y, int32_t ld, const float *t, float *dy,
                         double *loss, double *work, int64_t work_doubles, void *stream) {
    if (batch < 1 || n < 1 || ld < 1 || !y || !t || !loss || !work) return fail(KIFMM_EINVAL, "bad argument");
    const int64_t V = (int64_t)n * n * n;
    int nblk = (int)std::min<int64_t>(256, (V + 255) / 256);
    if ((int64_t)batch * (2 * nblk + 1) > work_doubles) return fail(KIFMM_EINVAL, "work space too small");
    double *part = work, *tn = work + (int64_t)batch * 2 * nblk;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(loss_partial_kernel, dim3(nblk, batch), dim3(kT), 0, st, n, V, y, ld, t, nblk, part);
    KIFMM_HIP(hipGetLastError());
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, batch, nblk, part, loss, tn);
    KIFMM_HIP(hipGetLastError());
    if (dy) {
        hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks((int64_t)batch * V)), dim3(kT), 0, st, n, V, batch, y, ld, t,
                           tn, dy);
        KIFMM_HIP(hipGetLastError());
    }
    return KIFMM_OK;
}

int kifmm_nn_adam(int64_t n, float *w, const float *g, float *m, float *v, int32_t step, float lr, float b1,
                  float b2, float eps, void *stream) {
    if (n < 0 || step < 1 || !w || !g || !m || !v) return fail(KIFMM_EINVAL, "bad argument");
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(n)), dim3(kT), 0, (hipStream_t)stream, n, w, g, m, v, lr, b1, b2,
                       eps, c1, c2);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_pack_input(int32_t batch, int32_t n, const float *grid, const float *scale, float *feat, void *stream) {
    if (batch < 1 || !pow2(n) || !grid || !feat) return fail(KIFMM_EINVAL, "bad argument");
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks((int64_t)batch * n * n * n)), dim3(kT), 0, (hipStream_t)stream,
                       batch, n, grid, scale, feat);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_unpack_output(int32_t batch, int32_t n, const float *y, int32_t ld, const float *scale, float *grid,
                           void *stream) {
    if (batch < 1 || !pow2(n) || ld < 1 || !y || !grid) return fail(KIFMM_EINVAL, "bad argument");
    hipLaunchKernelGGL(unpack_output_kernel, dim3(blocks((int64_t)batch * n * n * n)), dim3(kT), 0,
                       (hipStream_t)stream, batch, n, y, ld, scale, grid);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_max_abs(int32_t batch, int64_t per_sample, const float *x, float *out, int32_t reciprocal, float *work,
                     int64_t work_floats, void *stream) {
    if (batch < 1 || per_sample < 1 || !x || !out || !work) return fail(KIFMM_EINVAL, "bad argument");
    int nblk = (int)std::min<int64_t>(256, (per_sample + 255) / 256);
    if ((int64_t)batch * nblk > work_floats) return fail(KIFMM_EINVAL, "work space too small");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(max_abs_partial_kernel, dim3(nblk, batch), dim3(kT), 0, st, per_sample, x, nblk, work);
    KIFMM_HIP(hipGetLastError());
    hipLaunchKernelGGL(max_abs_final_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, batch, nblk, work, out,
                       reciprocal);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // extern "C"

// ------------------------------------------------ max |x| without a workspace --
// The partial maxima of kifmm_nn_max_abs_noalloc go to this file-scope device array
// instead of a caller's workspace.  Each GPU holds its own copy; host code reaches it only
// through the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[KIFMM_NN_MAX_ABS_SCRATCH];

namespace {
std::mutex g_scratch_mu;
std::vector<float *> g_scratch_ptr;   // per device ordinal, null until looked up

// device address of `scratch` on the current device, looked up once per device
int scratch_ptr(float **out) {
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= (int)g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        float *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KIFMM_OK;
}
}  // namespace

extern "C" {

int kifmm_nn_max_abs_noalloc(int32_t batch, int64_t per_sample, const float *x, float *out, int32_t reciprocal,
                             void *stream) {
    if (batch < 1 || per_sample < 1 || !x || !out) return fail(KIFMM_EINVAL, "bad argument");
    const int nblk = (int)std::min<int64_t>(256, (per_sample + 255) / 256);
    if ((int64_t)batch * nblk > KIFMM_NN_MAX_ABS_SCRATCH)
        return fail(KIFMM_EINVAL, "batch * blocks exceeds the static scratch (" +
                                      std::to_string(KIFMM_NN_MAX_ABS_SCRATCH) + " floats)");
    float *part = nullptr;
    KIFMM_TRY_(scratch_ptr(&part));
    hipStream_t st = (hipStream_t)stream;
    // every entry read by the final kernel is written by the partial kernel first: nothing
    // of a previous call's contents is read
    hipLaunchKernelGGL(max_abs_partial_kernel, dim3(nblk, batch), dim3(kT), 0, st, per_sample, x, nblk, part);
    KIFMM_HIP(hipGetLastError());
    hipLaunchKernelGGL(max_abs_final_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, batch, nblk, part, out,
                       reciprocal);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_coarsen2(int32_t batch, int32_t n_coarse, const float *fine, float *coarse, void *stream) {
    if (batch < 1 || n_coarse < 1 || !fine || !coarse) return fail(KIFMM_EINVAL, "bad argument");
    hipLaunchKernelGGL(coarsen2_kernel, dim3(blocks((int64_t)batch * n_coarse * n_coarse * n_coarse)), dim3(kT), 0,
                       (hipStream_t)stream, batch, n_coarse, fine, coarse);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_upsample2(int32_t batch, int32_t n_coarse, const float *coarse, float *fine, void *stream) {
    if (batch < 1 || n_coarse < 1 || !fine || !coarse) return fail(KIFMM_EINVAL, "bad argument");
    const int64_t nf = 2 * (int64_t)n_coarse;
    hipLaunchKernelGGL(upsample2_kernel, dim3(blocks((int64_t)batch * nf * nf * nf)), dim3(kT), 0,
                       (hipStream_t)stream, batch, n_coarse, coarse, fine);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_sampled_rel_err(int64_t n_tgt, const float *S, const int64_t *tgt, const double *ref, double scale,
                             double *out, void *stream) {
    if (n_tgt < 1 || !S || !tgt || !ref || !out) return fail(KIFMM_EINVAL, "bad argument");
    hipLaunchKernelGGL(sampled_err_kernel, dim3(1), dim3(kT), 0, (hipStream_t)stream, n_tgt, S, tgt, ref, scale, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_scale(int64_t n, float *x, float s, void *stream) {
    if (n < 0 || (n > 0 && !x)) return fail(KIFMM_EINVAL, "bad argument");
    if (n == 0) return KIFMM_OK;
    hipLaunchKernelGGL(scale_kernel, dim3(blocks(n)), dim3(kT), 0, (hipStream_t)stream, n, x, s);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_add(int64_t n, const float *x, float *y, void *stream) {
    if (n < 0 || (n > 0 && (!x || !y))) return fail(KIFMM_EINVAL, "bad argument");
    if (n == 0) return KIFMM_OK;
    hipLaunchKernelGGL(add_kernel, dim3(blocks(n)), dim3(kT), 0, (hipStream_t)stream, n, x, y);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

int kifmm_nn_sampled_rel_diff(int64_t n_tgt, const float *S, const float *R, const int64_t *tgt, double *out,
                              void *stream) {
    if (n_tgt < 1 || !S || !R || !tgt || !out) return fail(KIFMM_EINVAL, "bad argument");
    hipLaunchKernelGGL(sampled_diff_kernel, dim3(1), dim3(kT), 0, (hipStream_t)stream, n_tgt, S, R, tgt, out);
    KIFMM_HIP(hipGetLastError());
    return KIFMM_OK;
}

}  // extern "C"
