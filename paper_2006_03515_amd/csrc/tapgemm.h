// Launch description of the tap-GEMM engine (see tapgemm.hip).
#pragma once
#include "common.h"

namespace kifmm {

template <typename TA, typename TI, typename TO>
struct TapArgs {
    const TA *A;          // operators, op i at A + i * a_stride, row-major M x K
    const TA *A2;         // split-BF16: low parts of A (same layout), else unused
    int64_t a_stride;
    int M, K;             // padded rows / columns
    const TI *in;         // in[src * in_ld + k]
    const TI *in2;        // staged low-precision kernel: low parts of the split input
    const uint8_t *in_nz; // per input box: 0 if all its values are zero (null: unknown);
                          // the staged kernels skip taps whose sources are all zero
    const uint8_t *out_need;// per output box: 0 if its values are not wanted (null: all are);
                            // the staged kernels give a tile with no wanted box no taps
                            // (it is written as zeros, or left as is when accumulating)
    int64_t in_ld;
    TO *out;              // out[b * out_ld + row]
    int64_t out_ld;
    int mode;             // SrcMode
    int nl;               // boxes per axis of the source level (SRC_NBR)
    int zroots;           // SRC_NBR: cubes of nl^3 boxes stacked along z (0 or 1: independent samples)
    int nclass;           // number of output classes
    int cls_stride;       // output box = cls_stride * j + class
    int64_t n_per_class;
    int64_t n_boxes;      // nclass * n_per_class (size of the output in boxes)
    const int *tap_op;    // [nclass][ntaps]; null: use inl_op / inl_off
    const int *tap_off;   // [nclass][ntaps]
    int ntaps;
    int accumulate;       // 0: out = sum, 1: out += sum
    float *part;          // scratch for tap-group partial sums (may be null: no split)
    int64_t part_capacity;// floats available at part
    int groups;           // set by the launcher
    const float *amax;    // low precision: partial maxima of |in|
    int n_amax;
    float op_scale;       // low precision: A was stored divided by op_scale
    int pass;             // PASS_* below: selects a separately named kernel instance
    int inl_op[32];       // tap table passed by value (nclass * ntaps <= 32)
    int inl_off[32];
};

// Weight gradient of a tap GEMM: dW[t] (M x K) = sum_j dY[b_j] (M) . X[src_j]^T (K),
// b_j = cls_stride * j + cls(t), cls(t) = class_is_tap ? t : 0, src_j = src(b_j, t).
struct WgradArgs {
    const float *dy;      // dy[b * M + m]
    const float *x;       // x[src * K + k]
    float *dw;            // dw[t][M][K]
    int M, K;
    int mode, nl, cls_stride, class_is_tap;
    int64_t n_per_class;
    int ntaps;
    int tap_off[32];
    float *part;          // scratch for voxel-group partials
    int64_t part_capacity;
    int groups;           // set by the launcher
};

// Kernel instances are compiled once per pass kind so that profilers report the
// near field and the M2L translations under their own names.
enum { PASS_GENERIC = 0, PASS_P2P = 1, PASS_M2L = 2 };

int run_tap_f32(const TapArgs<float, float, float> &p, hipStream_t st);
int run_tap_f64(const TapArgs<double, double, double> &p, hipStream_t st);
template <typename TL>
int run_tap_lp(const TapArgs<TL, float, float> &p, bool x3, hipStream_t st);
int run_amax(const float *x, int64_t n, float *part, int nparts, hipStream_t st);
template <typename TL>
int run_split_lp(const float *x, int64_t n, const float *amax, int n_amax, TL *hi, TL *lo, hipStream_t st);
template <typename TL>
int run_tap_lp_staged(const TapArgs<TL, TL, float> &p, bool x3, hipStream_t st);
int run_wgrad(WgradArgs p, bool bf16, hipStream_t st);

}  // namespace kifmm
