/*
 * kifmm.h -- C ABI of libkifmm: kernel-independent fast multipole evaluation of
 * the 3D photoionization integral on one AMD Instinct MI355X (gfx950).
 *
 * What is computed (Lin, Zhuang, Cai, Zeng, Bao, "Accurate and efficient
 * calculation of photoionization in streamer discharges using fast multipole
 * method"):
 *
 *   Section 2.1, eq. (integral), (Ifun), (gfun):
 *     S_ph(x) = int I(y) g(|x-y|) / (4 pi |x-y|^2) dy,
 *     g(r)    = (exp(-chi_min pO2 r) - exp(-chi_max pO2 r)) / (r ln(chi_max/chi_min)).
 *   Section 3, eq. (summation) and the discrete kernel G after it: on a uniform
 *   grid of cell centres,
 *     S_i = prefactor * sum_j G(x_i, y_j) I_j (hx hy hz),
 *   G = g/(4 pi R^2) off the diagonal (midpoint rule) and
 *   G_ii = 3 g(rho) / (pi (hx^2+hy^2+hz^2)), rho = sqrt((hx^2+hy^2+hz^2)/12)
 *   (2x2x2 Gauss-Legendre rule on the self cell).
 *
 * kifmm_eval approximates that sum by the kernel-independent FMM of Section 3
 * (tree, upward pass eq. (s2m)/(m2m), downward pass eq. (m2l)/(l2l), target
 * potential = local expansion + near-range direct sum, eq. (nearfar)).
 * direct_eval computes the sum itself at chosen targets.
 *
 * Conventions
 *   Units: cm and Torr; chi in 1/(cm Torr).
 *   Arrays: C order [nx][ny][nz] (z fastest).  Cell (i,j,k) has centre
 *   (x0 + (i+1/2) hx, y0 + (j+1/2) hy, z0 + (k+1/2) hz).
 *   Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *   tensors); everything else is host memory that is read during the call only.
 *   stream: a hipStream_t passed as void*; NULL means the legacy default stream.
 *   Work is enqueued on `stream`; kifmm_eval and direct_eval return before it
 *   finishes, never synchronise the device, and allocate no memory.
 *   kifmm_eval forks its internal streams from `stream` and joins them back
 *   through events, so a call may be captured in a HIP graph on `stream`
 *   (replays repeat the evaluation on the same pointers; calls or replays that
 *   overlap on one ops object race).
 *   Inputs are never modified.
 *
 * Errors
 *   Every int-returning function returns KIFMM_OK (0) or a negative code, and
 *   never throws or aborts.  kifmm_last_error() returns a message for the last
 *   failure on the calling thread (thread-local storage, valid until the next
 *   failing call on that thread).
 */
#ifndef KIFMM_H
#define KIFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KIFMM_OK = 0,
    KIFMM_EINVAL = -1,       /* null pointer, non-positive size/spacing/pressure, bad option */
    KIFMM_EUNSUPPORTED = -2, /* valid request this library does not implement (e.g. non-cubic grid) */
    KIFMM_EMISMATCH = -3,    /* operators used with a tree they were not built for */
    KIFMM_ENOMEM = -4,       /* device allocation failed */
    KIFMM_EHIP = -5          /* a HIP runtime or rocBLAS call failed; the message names it */
};

/* Uniform grid of cell centres (Section 4: V = V' = a box of equal cells). */
typedef struct {
    int32_t nx, ny, nz;   /* cells per axis, > 0 */
    double x0, y0, z0;    /* lower corner [cm] */
    double hx, hy, hz;    /* cell sizes [cm], > 0 */
} kifmm_grid;

/* Kernel parameters of eq. (gfun): a = chi_min * p_o2, b = chi_max * p_o2.
 * The paper's values are chi_min = 0.035, chi_max = 2 (Section 2.1).
 * Requires 0 < chi_min < chi_max and p_o2 > 0. */
typedef struct {
    double chi_min, chi_max, p_o2;
} kifmm_kernel;

/* Placement of the equivalent and check points (Section 3: multipole and local
 * expansions, m0 points per side).  Radii are multiples of the box half-width r.
 *   KIFMM_LAYOUT_PAPER : one surface each, m0 per edge; upward equivalent at
 *                        1.05 r, upward check at 2.95 r, downward equivalent at
 *                        2.95 r, downward check at 1.05 r.
 *   KIFMM_LAYOUT_SINGLE: upward equivalent: m0 surface at 1.05 r; upward check:
 *                        surfaces at 2.95 r, 4 r, 6 r with check_edge points per
 *                        edge; downward equivalent: m0 surface at 2.95 r;
 *                        downward check: check_edge^3 lattice on [-1.05 r, 1.05 r]^3.
 *   KIFMM_LAYOUT_NESTED: as SINGLE plus a second m0 surface at 0.55 r (upward
 *                        equivalent) and at 4 r (downward equivalent).
 *   KIFMM_LAYOUT_LATTICE: upward equivalent and downward check: the full m0^3
 *                        lattice on [-R r, R r]^3, R = lattice_radius (0: 1.2;
 *                        0.5 < R <= 2; 3 <= m0 <= 8); upward check
 *                        as SINGLE; downward equivalent as NESTED.  Both M2L point
 *                        sets lie on lattices of one spacing, which lets M2L run in
 *                        its FFT form (kifmm_ops_m2l_fft; on by default).
 * rcond: singular values <= rcond * s_max are dropped from the pseudo-inverse.
 * Expansions are carried as coefficients on the retained left singular vectors
 * of the check-to-equivalent matrix (the backward-stable form of the
 * pseudo-inverse, Section 3 remark on the pseudo-inverse). */
enum { KIFMM_LAYOUT_PAPER = 0, KIFMM_LAYOUT_SINGLE = 1, KIFMM_LAYOUT_NESTED = 2, KIFMM_LAYOUT_LATTICE = 3 };
typedef struct {
    int32_t layout;       /* KIFMM_LAYOUT_* */
    int32_t m0;           /* equivalent points per cube edge, 2..16 (paper: 6) */
    int32_t check_edge;   /* check points per edge, layouts SINGLE/NESTED/LATTICE, 2..16 */
    double rcond;         /* relative SVD cutoff, 0 < rcond < 1 */
    double lattice_radius;/* layout LATTICE: lattice half-width / r (0: 1.2); else ignored */
} kifmm_opts;

/* Arithmetic of kifmm_eval.
 *   KIFMM_FP64      : all passes in FP64; I_dev and S_dev are double*.
 *   KIFMM_FP32      : all passes in FP32 (FP32 MFMA); float* I/O.
 *   KIFMM_M2L_BF16  : as FP32 but the M2L translations take bfloat16 operands
 *                     (FP32 accumulate); float* I/O.
 *   KIFMM_M2L_FP16  : as FP32 but M2L in FP16 operands; operators and inputs
 *                     are scaled by their maximum magnitude per level.
 *   KIFMM_M2L_BF16X3: as FP32 but M2L in split bfloat16: each operand is the sum
 *                     of two bfloat16 numbers (high part + rounding residual)
 *                     and three bfloat16 products are accumulated in FP32
 *                     (about 16 significant bits per operand).
 *   KIFMM_BF16X3    : the near field (P2P), M2L and, on leaves of 8^3 cells,
 *                     P2M and L2P (fused with the permutes) in split bfloat16;
 *                     the near-range matrices, self cell included, and the
 *                     leaf operators are computed in FP64 and then split.
 *                     Other passes FP32.
 *   KIFMM_BF16      : every translation GEMM (P2M, M2M, M2L, L2L, L2P) with
 *                     bfloat16 operands, FP32 accumulation: operators stored
 *                     divided by their maxima, inputs divided by theirs; the
 *                     near field and its self cell in FP32 (operators and
 *                     pseudo-inverses built in FP64).
 *   KIFMM_FP16      : the same with FP16 operands.
 * With kifmm_ops_p2p_fft on, the near field of every single-precision mode other
 * than a dense KIFMM_BF16X3 runs in Fourier space (FP32). */
enum { KIFMM_FP64 = 0, KIFMM_FP32 = 1, KIFMM_M2L_BF16 = 2, KIFMM_M2L_FP16 = 3, KIFMM_M2L_BF16X3 = 4,
       KIFMM_BF16X3 = 5, KIFMM_BF16 = 6, KIFMM_FP16 = 7 };

typedef struct kifmm_tree_s *kifmm_tree;
typedef struct kifmm_ops_s *kifmm_ops;

/* Tree construction (Section 3, step 1 of the algorithm outline; its closing remark on
 * non-uniform meshes for cells with hz != hx).
 * Cubic grid of cubic cells (nx == ny == nz = 2^p, hx == hy == hz): the complete octree
 * whose leaves are cubes of ell^3 cells, ell^3 <= max_leaf (the paper's m) with ell the
 * largest power of two that fits.
 * Box nx == ny = 2^p, nz, with hx == hy and any hz: leaves of ell x ell x ellz cells,
 * ellz the power of two closest to ell hx / hz (leaves nearly cubic in space), ell the
 * largest power of two with ell^2 ellz <= max_leaf; the leaves form a column of R root
 * cubes of (nx / ell)^3 leaves along z, each a complete octree (nz must equal
 * R ellz nx / ell, R <= 64), and the near and far fields cross from one cube into the next
 * (at level 0 the roots two or more apart interact through M2L).
 * The leaf order (Morton within a root, root after root) is computed on the device.
 * Requires ell >= 4; otherwise KIFMM_EUNSUPPORTED; KIFMM_EINVAL for bad sizes or
 * max_leaf < 1.  Other box shapes of cubic cells are evaluated exactly inside the smallest
 * cube with zero sources outside the box (caller-side: paper_2006_03515_amd/embedding.py).
 * Allocates device memory owned by the tree; *out is set only on success.  Synchronises
 * `stream` before returning. */
int kifmm_build_tree(const kifmm_grid *grid, int32_t max_leaf, void *stream, kifmm_tree *out);

/* Operator precompute for one tree and one pressure (Section 3, eq. (s2m),
 * (s2l), (m2m), (m2l), (l2l)).  In FP64 on the device: kernel matrices between
 * point sets, truncated SVD (one-sided Jacobi) of the check-to-equivalent
 * matrices of every level, the fused translation operators, the near-range
 * matrices with the self-cell value; then FP32/BF16/FP16 copies.  Allocates
 * device memory owned by the returned object.  Synchronises `stream`.
 * opts may be NULL (defaults: SINGLE, m0 = 6, check_edge = 10, rcond = 1e-7). */
int kifmm_precompute_operators(kifmm_tree tree, const kifmm_kernel *kernel,
                               const kifmm_opts *opts, void *stream, kifmm_ops *out);

/* Retained SVD ranks of level `level` (lmin <= level <= depth; lmin = 2 on a cube, 1 on a column of
 * two cubes, 0 on a column of three or more); returns 0 and
 * writes k_up/k_down, or a negative code. depth is returned by kifmm_tree_info. */
int kifmm_ops_rank(kifmm_ops ops, int32_t level, int32_t *k_up, int32_t *k_down);

/* Tree shape: depth D (levels 0..D below each root), leaf side ell in cells (along x, y). */
int kifmm_tree_info(kifmm_tree tree, int32_t *depth, int32_t *leaf_side);
/* Leaf cells along x and y (ell) and along z (ellz), and the number R of root cubes along z
 * (1 for a cubic grid).  Any output pointer may be NULL. */
int kifmm_tree_shape(kifmm_tree tree, int32_t *leaf_xy, int32_t *leaf_z, int32_t *roots);

/* FMM evaluation: S_dev[i] ~= prefactor * sum_j G(x_i,y_j) I_dev[j] hx hy hz for
 * every cell i.  I_dev and S_dev hold nx*ny*nz values, double for KIFMM_FP64 and
 * float otherwise, in grid order; they must not overlap.  `ops` must come from
 * `tree` (else KIFMM_EMISMATCH).  Uses the work buffers owned by `ops`, so
 * calls sharing one ops object must be ordered on one stream.  The near field
 * (and, after it, the M2L of the coarse levels D-1 .. 4 when both Fourier forms are on)
 * runs on a second stream, the finest level's FFT-form M2L on a third and level 3's on
 * a fourth; the library creates these three once per device and shares them between all
 * operator objects (kept until the process ends), and all are forked from and joined
 * back into `stream` with events, so when the call returns, all its work is ordered on
 * `stream` (also when it returns an error).  Evaluations of different ops objects may be
 * issued on different streams; their side work then shares the three streams.  With
 * leaves of 8^3 cells and FP32 arithmetic, P2M runs fused with the permute of I into
 * leaf order and L2P fused with the sum of far and near field and the permute back
 * (16-byte aligned I_dev and S_dev; otherwise separate permutes and tap GEMMs). */
int kifmm_eval(kifmm_tree tree, kifmm_ops ops, const void *I_dev, double prefactor,
               void *S_dev, int32_t precision, void *stream);

/* Zero-source skipping (an addition to the method: it changes which terms are
 * added, not their values).  With enable != 0, every later kifmm_eval with these
 * ops marks the leaves whose sources are all exactly zero and the boxes all of whose
 * leaves are marked (one pass over the leaf-ordered sources, before the near field
 * starts), and the near field, P2M, M2M and M2L skip, per output tile of 64 boxes,
 * the taps whose source boxes are all marked.  The skipped terms are exact zeros, so
 * the result is the same sum; the FP32 partial sums are grouped differently, which
 * changes results at rounding level.  It pays for sources that vanish on large
 * regions (localized sources, a box-shaped grid embedded in a cube) and costs the
 * marking pass otherwise.  The first enable allocates one byte per box of levels
 * 2..D, owned by ops; enable = 0 turns skipping off.  FP64 evaluations and trees of
 * depth < 2 are unaffected.  Returns 0, KIFMM_EINVAL (ops NULL) or KIFMM_ENOMEM. */
int kifmm_ops_skip_zero_sources(kifmm_ops ops, int32_t enable);

/* Target restriction: evaluation on a part of the domain only (Section 5.1, closing
 * remark: S_ph is often needed on a sub-region).  leaf_mask is a host array of
 * nb * nb * (R nb) bytes, nb = n / ell leaves per axis of a root cube (ell, R from
 * kifmm_tree_shape), in C order [nb][nb][R nb] over leaf coordinates (leaf (a, b, c) holds
 * the cells a*ell .. a*ell+ell-1 along x, and c*ellz .. along z); nonzero marks a wanted
 * leaf.  It is copied (the caller keeps
 * ownership).  Every later kifmm_eval with these ops returns, at each cell of a wanted
 * leaf, exactly what it returns without the restriction (bit for bit: the sum and its
 * order are unchanged), and 0 at every other cell.  M2L, L2L, L2P and the near field
 * skip, per output tile of 64 boxes, the tiles that hold no box with a wanted leaf
 * below it; the upward pass is unchanged.  leaf_mask = NULL removes the restriction.
 * The call synchronizes the device (flags in use by an evaluation are not
 * overwritten).  Returns 0, KIFMM_EINVAL (ops NULL), KIFMM_ENOMEM or KIFMM_EHIP. */
int kifmm_ops_restrict_targets(kifmm_ops ops, const uint8_t *leaf_mask);

/* FFT form of M2L (Section 3 remark: the translation between equivalent and check
 * points on regular grids is a convolution).  Operators built with
 * KIFMM_LAYOUT_LATTICE hold, per level, the spectra of the kernel on the
 * (2 m0 - 1)^3 cyclic grid for the 316 offsets and the maps between coefficients
 * and lattice values (W_u, U_d^T).  With enable != 0 (the default for that layout),
 * the M2L of KIFMM_FP32, KIFMM_BF16X3, KIFMM_M2L_BF16X3, KIFMM_M2L_FP16 and
 * KIFMM_M2L_BF16 evaluations runs as: equivalent densities on the lattice (FP32 MFMA
 * GEMM), their half spectra (separable DFT), per frequency the products with the kernel
 * spectra over each box's interaction list (grouped by parents into one 16 x 432 real
 * matrix per frequency: FP32 MFMA; split bfloat16 MFMA for the two BF16X3 modes; single
 * FP16 or bfloat16 operands for KIFMM_M2L_FP16 / KIFMM_M2L_BF16, each frequency's matrix
 * and each workgroup's spectra scaled by powers of two into FP16's range), check
 * potentials on the lattice (separable inverse DFT) and coefficients (FP32 MFMA GEMM).
 * The levels with fewer than 4 parents per axis keep the products in FP32.  FP32
 * computes the same sum as the dense M2L of the same layout up to FP32 rounding;
 * enable = 0 selects the dense M2L (FP64, KIFMM_BF16 and KIFMM_FP16 always use it).
 * Returns 0,
 * KIFMM_EINVAL (ops NULL) or KIFMM_EUNSUPPORTED (another layout). */
int kifmm_ops_m2l_fft(kifmm_ops ops, int32_t enable);

/* Near field in Fourier space (eq. (nearfar), direct part, with the self cell).  On the
 * uniform grid the matrix between a leaf of 8^3 cells and a neighbour leaf is a block of a
 * convolution, so with enable != 0 the near field of every single-precision evaluation
 * runs as: half spectra (15 x 15 x 8) of every leaf's sources zero-padded to 15^3,
 * 27 complex products per frequency against the kernel spectra of the 27 neighbour
 * offsets (built in FP64 with the operators; the frequencies that are conjugates of others
 * are neither stored nor multiplied), and the inverse transform at the 8^3 cells.
 * Same sum as the dense near field up to FP32 rounding (about 1e-7 of the result).  The
 * first enable allocates spectra buffers of 22.5 KiB per leaf (owned by ops).  Returns
 * 0, KIFMM_EINVAL (ops NULL), KIFMM_EUNSUPPORTED (leaves other than 8^3, or fewer than 4
 * per axis) or KIFMM_ENOMEM. */
int kifmm_ops_p2p_fft(kifmm_ops ops, int32_t enable);

/* Direct evaluation of the exact sum (Section 3, eq. (summation)):
 * out_dev[t] = prefactor * sum_j G(x_t, y_j) I_dev[j] hx hy hz for the flat cell
 * indices tgt_idx_dev[t] (device int64, each in [0, N)), or for every cell
 * t = 0..N-1 when tgt_idx_dev is NULL (then n_tgt must equal N).  I_dev is float
 * [N]; out_dev is double [n_tgt].  fp64_accumulate = 1 evaluates the kernel in
 * FP64; 0 evaluates it in FP32 (distances from integer cell offsets, 1/R from the
 * hardware reciprocal square root, exponentials from the hardware base-2
 * exponential, 1 - e^{-x} from a series below x = 1/2; per-value relative error
 * about 1e-7).  Sums are
 * always FP64, in a fixed order (bitwise repeatable).  Any grid is accepted.
 * n_tgt = 0 is a no-op (out_dev may then be NULL).  Out-of-range indices are
 * not checked on the device: the caller guarantees them. */
int direct_eval(const kifmm_grid *grid, const kifmm_kernel *kernel, const float *I_dev,
                double prefactor, const int64_t *tgt_idx_dev, int64_t n_tgt,
                double *out_dev, int32_t fp64_accumulate, void *stream);

/* Morton leaf order of the tree: perm_dev[p] = grid index of the cell stored at
 * position p of the leaf-ordered layout (int64 [N], device).  For tests. */
int kifmm_tree_permutation(kifmm_tree tree, int64_t *perm_dev, void *stream);

/* Per-pass timing of kifmm_eval (instrumentation for benchmarks).
 * kifmm_profile_enable(ops, 1) creates HIP events (on the current device) and
 * from then on every kifmm_eval with `ops` records an event pair around each
 * pass on the evaluation stream; (ops, 0) stops recording and clears the sums.
 * kifmm_profile_read synchronises those events and returns, for each pass
 * p < n (KIFMM_PASS_*), the summed elapsed milliseconds ms[p] and the number of
 * kernel launches calls[p] since enabling (either array may be NULL).  While
 * profiling is on, kifmm_eval may wait for old events when the event pool
 * (4096 pairs) is nearly full; with profiling off it never waits. */
enum { KIFMM_PASS_PERMUTE_IN = 0, KIFMM_PASS_P2M = 1, KIFMM_PASS_M2M = 2, KIFMM_PASS_M2L = 3,
       KIFMM_PASS_L2L = 4, KIFMM_PASS_L2P = 5, KIFMM_PASS_P2P = 6, KIFMM_PASS_PERMUTE_OUT = 7,
       KIFMM_PASS_NEAR_PRODUCTS = 8, /* inside P2P: the products of the Fourier-space near field */
       KIFMM_NPASS = 9 };
int kifmm_profile_enable(kifmm_ops ops, int32_t on);
int kifmm_profile_read(kifmm_ops ops, double *ms, int64_t *calls, int32_t n);

/* Serial schedule (measurement).  With enable != 0, every later kifmm_eval with `ops`
 * runs all its passes on the calling stream, one after the other (near field first,
 * then the upward pass, M2L level by level and the downward pass), instead of forking
 * the near field and the M2L of the finest and coarse levels onto the library's own
 * streams.  The results are bit for bit those of the concurrent schedule (the same
 * kernels on the same data); only the overlap is lost, so each kernel's duration in a
 * trace is its own.  Returns 0 or KIFMM_EINVAL (ops NULL). */
int kifmm_ops_serial(kifmm_ops ops, int32_t enable);

/* ------------------------------------------------------------------------
 * Learned surrogate (not in the paper): kernels of a 3D convolutional network
 * that maps a coarse source field to S_ph, trained on pairs made by kifmm_eval
 * and used with kifmm_eval / direct_eval as judge and fallback.
 *
 * Activations: FP32, channels-last, voxels of an n^3 grid (n a power of two) in
 * Morton order per sample: x[(s * n^3 + morton(i, j, k)) * C + c].  Weights:
 * FP32 masters [taps][co][ci]; the layer kernels read copies made by
 * kifmm_nn_prepare_weights (FP32 or BF16, forward [taps][co][ci] and transposed
 * [taps][ci][co] for the data gradient).  bf16 = 1 runs the products on BF16
 * MFMA with FP32 accumulation (inputs rounded to nearest-even when staged);
 * bf16 = 0 on FP32 MFMA.  Products of one output are summed in FP32 over at
 * most 8 MFMA steps and then in FP64.
 * Layer kinds (taps in C order):
 *   KIFMM_NN_CONV3  3x3x3 stride 1 zero padding, 27 taps (dz, dy, dx) in {-1,0,1}^3
 *   KIFMM_NN_DOWN2  2x2x2 stride 2 (n -> n/2), 8 taps = child parity (pz, py, px)
 *   KIFMM_NN_UP2    transposed 2x2x2 stride 2 (n -> 2n), 8 taps = child parity
 *   KIFMM_NN_POINT  1x1x1
 * n_in is the grid side of the layer input.  ci (the reduction) must be a
 * multiple of 32 and co a multiple of 16 (32 for the weight gradient).
 * work / work_floats: optional device scratch for split reductions (the calls
 * allocate nothing; with too little scratch they use fewer workgroups).
 * All calls enqueue on `stream` and return before the work ends. */
enum { KIFMM_NN_CONV3 = 0, KIFMM_NN_DOWN2 = 1, KIFMM_NN_UP2 = 2, KIFMM_NN_POINT = 3 };
/* y (+)= layer(x) */
int kifmm_nn_layer_forward(int32_t kind, int32_t batch, int32_t n_in, const float *x, int32_t ci,
                           const void *w, int32_t co, float *y, int32_t accumulate, int32_t bf16,
                           float *work, int64_t work_floats, void *stream);
/* dx (+)= layer^T(dy) with the transposed weights wt [taps][ci][co] */
int kifmm_nn_layer_backward_data(int32_t kind, int32_t batch, int32_t n_in, const float *dy, int32_t co,
                                 const void *wt, int32_t ci, float *dx, int32_t accumulate, int32_t bf16,
                                 float *work, int64_t work_floats, void *stream);
/* dw [taps][co][ci] = dL/dw given the layer input x and dL/dy (overwritten) */
int kifmm_nn_layer_backward_weight(int32_t kind, int32_t batch, int32_t n_in, const float *x, int32_t ci,
                                   const float *dy, int32_t co, float *dw, int32_t bf16, float *work,
                                   int64_t work_floats, void *stream);
/* w_fwd = cast(w) [taps][co][ci], w_bwd = cast(w)^T [taps][ci][co] (either may be NULL) */
int kifmm_nn_prepare_weights(int32_t taps, int32_t co, int32_t ci, const float *w, void *w_fwd,
                             void *w_bwd, int32_t bf16, void *stream);
/* y = leaky(y + bias) in place (bias [c] or NULL; alpha = 1 gives the identity) */
int kifmm_nn_bias_act(int64_t nvox, int32_t c, float *y, const float *bias, float alpha, void *stream);
/* dy <- dy * leaky'(.) (using the sign of the post-activation y) and dbias = sum of
 * the result over voxels (fixed-order reduction; work >= min(1024, nvox/256) * c floats) */
int kifmm_nn_bias_act_backward(int64_t nvox, int32_t c, const float *y, float *dy, float *dbias,
                               float alpha, float *work, int64_t work_floats, void *stream);
/* Squared relative L2 loss of channel 0 of y (Morton, row length ld) against the
 * grid-ordered target t, per sample, averaged over the batch: loss[0] = mean,
 * loss[1 + s] = per sample (double, device).  dy (optional, layout of y) gets
 * dL/dy (zero outside channel 0).  work >= batch * (2 * min(256, n^3/256) + 1) doubles. */
int kifmm_nn_rel_l2_loss(int32_t batch, int32_t n, const float *y, int32_t ld, const float *t, float *dy,
                         double *loss, double *work, int64_t work_doubles, void *stream);
/* Adam step `step` (>= 1) on n FP32 master weights */
int kifmm_nn_adam(int64_t n, float *w, const float *g, float *m, float *v, int32_t step, float lr,
                  float b1, float b2, float eps, void *stream);
/* network input: 27-neighbourhood of scale[s] * grid[s] (grid order) as 32 channels
 * (the last 5 zero) in Morton order; scale may be NULL (1) */
int kifmm_nn_pack_input(int32_t batch, int32_t n, const float *grid, const float *scale, float *feat,
                        void *stream);
/* grid[s][g] = scale[s] * y[(s n^3 + morton(g)) * ld] (channel 0) */
int kifmm_nn_unpack_output(int32_t batch, int32_t n, const float *y, int32_t ld, const float *scale,
                           float *grid, void *stream);
/* out[s] = max |x_s| over per_sample values, or its reciprocal (1 for a zero field) */
int kifmm_nn_max_abs(int32_t batch, int64_t per_sample, const float *x, float *out, int32_t reciprocal,
                     float *work, int64_t work_floats, void *stream);
/* kifmm_nn_max_abs for callers that cannot allocate device memory (code under stream
 * capture, serving loops that must not call hipMalloc): the same result, with the
 * per-block partial maxima kept in a static device array of KIFMM_NN_MAX_ABS_SCRATCH
 * floats (1 MiB) instead of a caller's workspace.  Each GPU the library runs on holds its
 * own copy of that array until the process ends; its address on a device is looked up
 * (hipGetSymbolAddress) on the first call made with that device current.  Nothing is
 * allocated.  batch * min(256, ceil(per_sample / 256)) must not exceed
 * KIFMM_NN_MAX_ABS_SCRATCH, else KIFMM_EINVAL before any device work.  All calls on one GPU
 * share the array and leave their partial maxima in it: calls that overlap on one GPU
 * (other streams, other host threads) race and must be ordered by the caller.  Returns 0,
 * KIFMM_EINVAL or KIFMM_EHIP. */
#define KIFMM_NN_MAX_ABS_SCRATCH 262144
int kifmm_nn_max_abs_noalloc(int32_t batch, int64_t per_sample, const float *x, float *out, int32_t reciprocal,
                             void *stream);
/* 2x2x2 block means of a (2 n_coarse)^3 grid-ordered field */
int kifmm_nn_coarsen2(int32_t batch, int32_t n_coarse, const float *fine, float *coarse, void *stream);
/* trilinear interpolation from cell centres of an n_coarse^3 field to those of the
 * (2 n_coarse)^3 field, clamped at the boundary */
int kifmm_nn_upsample2(int32_t batch, int32_t n_coarse, const float *coarse, float *fine, void *stream);
/* out[0] = ||scale * S[tgt] - ref|| / ||ref|| (one workgroup, fixed order) */
int kifmm_nn_sampled_rel_err(int64_t n_tgt, const float *S, const int64_t *tgt, const double *ref,
                             double scale, double *out, void *stream);
/* x[0:n] *= s (a prediction made for prefactor 1, rescaled) */
int kifmm_nn_scale(int64_t n, float *x, float s, void *stream);
/* y[0:n] += x[0:n] (the gradient of a skip connection's source, summed over its two uses) */
int kifmm_nn_add(int64_t n, const float *x, float *y, void *stream);
/* out[0] = ||S[tgt] - R[tgt]|| / ||R[tgt]|| for two FP32 fields in grid order (one workgroup,
 * FP64 sums in a fixed order): the serving check of a prediction S against a judge's field R */
int kifmm_nn_sampled_rel_diff(int64_t n_tgt, const float *S, const float *R, const int64_t *tgt, double *out,
                              void *stream);

void kifmm_tree_destroy(kifmm_tree tree);  /* NULL is ignored */
void kifmm_ops_destroy(kifmm_ops ops);     /* NULL is ignored */
const char *kifmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KIFMM_H */
