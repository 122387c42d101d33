// C ABI of libkifmm: argument checking, tree and operator objects, the
// precompute orchestration and the evaluation schedule (Section 3, algorithm
// outline: tree, upward pass, downward pass, target potential).
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "common.h"
#include "tapgemm.h"

namespace kifmm {

// ------------------------------------------------------------------ errors --
static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
int fail(int code, const std::string &m) {
    g_err = m;
    return code;
}
int hip_fail(hipError_t e, const char *what) {
    g_err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return KIFMM_EHIP;
}

// launchers defined in the other translation units
int launch_direct(const kifmm_grid *, const kifmm_kernel *, const float *, double, const int64_t *,
                  int64_t, double *, int, hipStream_t);
int launch_morton_scatter(const Tree &, hipStream_t);
template <typename T> int launch_permute_in(const Tree &, const T *, T, T *, hipStream_t);
template <typename T> int launch_permute_out(const Tree &, const T *, T, const uint8_t *, T *, hipStream_t);
int launch_perm_i64(const Tree &, int64_t *, hipStream_t);
int launch_kmat(const double *, int, const double *, int, const double *, const double *, int, int,
                const kifmm_kernel &, double, double *, hipStream_t);
int launch_near(int, int, double, double, const int *, int, const kifmm_kernel &, double *, hipStream_t);
int launch_jacobi_round(double *, double *, const int *, const int *, int, int, int, int64_t,
                        int64_t, int, int, double, unsigned long long *, hipStream_t);
int launch_colnorm(const double *, const int *, const int *, int, int64_t, int, int, double *,
                   hipStream_t);
int launch_svd_gather(const double *, const double *, int, int, int, int, int, const int *,
                      const double *, double *, double *, hipStream_t);
int launch_gemm_f64(int, int, int, const double *, int, int64_t, const double *, int, int64_t,
                    double *, int, int64_t, int, hipStream_t);
template <typename T>
int launch_cast_pad(const double *, int, int, int64_t, T *, int, int, int64_t, int, double,
                    hipStream_t);
int launch_cast_pad_lo(const double *, int, int, int64_t, __bf16 *, int, int, int64_t, int, double,
                       hipStream_t);
int run_m2l_hadamard(const float *, const float *, const int *, const int *, int, int, int, const uint8_t *,
                     const uint8_t *, float *, hipStream_t);
int run_m2l_pair_mfma(const float *, const float *, int, int, const uint8_t *, const uint8_t *, float *, hipStream_t);
int run_m2l_pair_bf16x3(const float *, const float *, int, int, const uint8_t *, const uint8_t *, float *, hipStream_t);
int run_m2l_pair_lp1(int, const float *, const void *, const float *, int, int, const uint8_t *, const uint8_t *, float *,
                     hipStream_t);
int run_m2l_lattice(int, int, const float *, int64_t, int, int, const uint8_t *, float *, hipStream_t);
int run_near_fft_stage(int, const float *, const float *, int, const uint8_t *, const uint8_t *, float *, float *,
                       float *, hipStream_t, const float *, float);
template <typename T>
int launch_permute_out2(const Tree &, const T *, const T *, T, const uint8_t *, T *, hipStream_t);
int launch_pack_fragments(const float *, int, int, int, int, float4 *, hipStream_t);
int l2p_fragment_chunks(int KD);
bool leafgemm_fits(const Tree &, int, int);
int run_p2m_permute_in(const Tree &, const float *, float, const float4 *, int, float *, float *, hipStream_t);
int run_l2p_permute_out(const Tree &, const float *, int, const float4 *, const float *, float, const uint8_t *, float *,
                        hipStream_t);
int launch_pack_fragments_x3(const double *, int, int, int, int, uint4 *, hipStream_t);
int l2p_fragment_chunks_x3(int KD);
int run_p2m_permute_in_x3(const Tree &, const float *, float, const uint4 *, int, float *, float *, hipStream_t);
int run_l2p_permute_out_x3(const Tree &, const float *, int, const uint4 *, const float *, float, const uint8_t *,
                           float *, hipStream_t);

static std::atomic<uint64_t> g_magic{0x6b69666d6d000001ull};

template <typename T>
static int dmalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return KIFMM_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(KIFMM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                      " bytes failed: " + hipGetErrorString(e));
    }
    return KIFMM_OK;
}

#define KIFMM_TRY(x)                 \
    do {                             \
        int rc_ = (x);               \
        if (rc_ != KIFMM_OK) return rc_; \
    } while (0)

static int pad_to(int v, int m) { return (v + m - 1) / m * m; }

// ------------------------------------------------------------- point sets --
// Points of an m x m x m lattice on [-rad, rad]^3 lying on its boundary.
static void cube_surface(int m, double rad, std::vector<double> &out) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < m; ++k) {
                if (!(i == 0 || j == 0 || k == 0 || i == m - 1 || j == m - 1 || k == m - 1)) continue;
                const double t = 2.0 * rad / (m - 1);
                out.push_back(-rad + i * t);
                out.push_back(-rad + j * t);
                out.push_back(-rad + k * t);
            }
}
static void cube_lattice(int m, double rad, std::vector<double> &out) {
    const double t = 2.0 * rad / (m - 1);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < m; ++k) {
                out.push_back(-rad + i * t);
                out.push_back(-rad + j * t);
                out.push_back(-rad + k * t);
            }
}
struct PointSets {
    std::vector<double> yu, xu, yd, xd;  // xyz triples, relative to the box centre
};
static PointSets make_point_sets(const kifmm_opts &o, double r) {
    PointSets p;
    if (o.layout == KIFMM_LAYOUT_PAPER) {
        cube_surface(o.m0, 1.05 * r, p.yu);
        cube_surface(o.m0, 2.95 * r, p.xu);
        cube_surface(o.m0, 2.95 * r, p.yd);
        cube_surface(o.m0, 1.05 * r, p.xd);
        return p;
    }
    for (double f : {2.95, 4.0, 6.0}) cube_surface(o.check_edge, f * r, p.xu);
    cube_lattice(o.check_edge, 1.05 * r, p.xd);
    cube_surface(o.m0, 1.05 * r, p.yu);
    cube_surface(o.m0, 2.95 * r, p.yd);
    if (o.layout == KIFMM_LAYOUT_NESTED || o.layout == KIFMM_LAYOUT_LATTICE) cube_surface(o.m0, 4.0 * r, p.yd);
    if (o.layout == KIFMM_LAYOUT_NESTED) cube_surface(o.m0, 0.55 * r, p.yu);
    if (o.layout == KIFMM_LAYOUT_LATTICE) {   // both M2L point sets on one lattice
        p.yu.clear();
        p.xd.clear();
        cube_lattice(o.m0, o.lattice_radius * r, p.yu);
        cube_lattice(o.m0, o.lattice_radius * r, p.xd);
    }
    return p;
}

static int pack_off(int x, int y, int z) { return ((x + 16) << 10) | ((y + 16) << 5) | (z + 16); }

// the 316 offsets of possible interaction-list members: [-3,3]^3 minus [-1,1]^3
static std::vector<int> m2l_offsets() {
    std::vector<int> o;
    for (int x = -3; x <= 3; ++x)
        for (int y = -3; y <= 3; ++y)
            for (int z = -3; z <= 3; ++z)
                if (std::max({std::abs(x), std::abs(y), std::abs(z)}) >= 2) {
                    o.push_back(x);
                    o.push_back(y);
                    o.push_back(z);
                }
    return o;
}

static int floordiv2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

}  // namespace kifmm

using namespace kifmm;

// ---------------------------------------------------------------- ops type --
struct kifmm_ops_s {
    uint64_t tree_magic = 0;
    int D = 0, ell = 0, s = 0, nb = 0;
    int ellz = 0, R = 1;               // leaf cells along z, root cubes along z
    int lmin = 2;                      // coarsest level with expansions: 2 on a cube, 1 on a column of 2, else 0
    // M2L of level 0 on a column of R > 2 cubes: the roots two or more apart, offsets
    // (0, 0, dz), 2 <= |dz| <= R - 1 (n0 operators)
    int n0 = 0;
    float *m2l0_32 = nullptr;
    double *m2l0_64 = nullptr;
    int KU = 0, KD = 0;
    std::vector<int> ku, kd;           // retained ranks per level
    kifmm_kernel kern{};
    kifmm_opts opts{};
    // operators
    float *p2m32 = nullptr, *m2m32 = nullptr, *m2l32 = nullptr, *l2l32 = nullptr, *l2p32 = nullptr,
          *p2p32 = nullptr;
    double *p2m64 = nullptr, *m2m64 = nullptr, *m2l64 = nullptr, *l2l64 = nullptr,
           *l2p64 = nullptr, *p2p64 = nullptr;
    __bf16 *m2lbf = nullptr, *m2lbf_lo = nullptr;   // split BF16: high and low parts
    __bf16 *p2pbf = nullptr, *p2pbf_lo = nullptr;
    float p2p_scale = 1.0f;            // max |near-range matrix entry| (split BF16 storage divisor)
    float *amax_q = nullptr;           // partial maxima of |q| (split BF16 near field)
    // split low-precision copies of the inputs of the staged kernels, high parts then
    // low parts: of q (near field, side stream) and of one level's multipole
    // coefficients (M2L, main stream)
    uint16_t *split_q = nullptr, *split_c = nullptr;
    int64_t split_q_n = 0, split_c_n = 0;   // elements per part
    // zero-source skipping (kifmm_ops_skip_zero_sources): per level l = 2..D, one byte per
    // box, 1 if some leaf below it has a nonzero source (level D: the leaves themselves)
    bool skip_zero = false;
    std::vector<uint8_t *> nz;
    // target restriction (kifmm_ops_restrict_targets): per level l = 0..D, one byte per box,
    // 1 if some leaf below it is wanted (level D: the leaves); empty: every target is wanted
    std::vector<uint8_t *> want;
    _Float16 *m2lh = nullptr;
    // KIFMM_BF16 / KIFMM_FP16: the surface operators (P2M, M2M per level, L2L per level, L2P)
    // stored divided by their maxima in BF16 and FP16
    __bf16 *p2mbf = nullptr, *m2mbf = nullptr, *l2lbf = nullptr, *l2pbf = nullptr;
    _Float16 *p2mh = nullptr, *m2mh = nullptr, *l2lh = nullptr, *l2ph = nullptr;
    float p2m_scale = 1.f, l2p_scale = 1.f;
    std::vector<float> m2m_scale, l2l_scale;   // per level (M2M: target level, L2L: target level)
    // FFT form of M2L (layout LATTICE): per level l, the kernel spectra of the 316 offsets
    // (fft_g[l], 316 x nfp complex), upward coefficients -> equivalent densities on the
    // lattice (lat_w[l] = W_u, lrow x KU, rows past m0^3 zero) and lattice check potentials
    // -> downward coefficients (lat_u[l] = U_d^T, KD x lrow), lrow = m0^3 padded to 32,
    // mf = 2 nfp; lattice values of the finest level (lat_buf: boxes of level D x lrow) and
    // its spectra (spec_e, spec_p: boxes of level D x mf), and the same for each coarser
    // level (the _c buffers: levels 2 .. D - 1 one after the other, (8^l - 64) / 7 boxes
    // before level l), since levels run at the same time on different streams
    bool m2l_fft = false;
    int nfp = 0, mf = 0, lrow = 0;
    std::vector<float *> fft_g, lat_w, lat_u;
    float *lat_buf = nullptr, *lat_buf_c = nullptr, *spec_e_c = nullptr, *spec_p_c = nullptr;
    std::vector<float *> fft_pair;   // levels with >= 8 boxes per axis: [nfp][27][64][4] MFMA fragments
    std::vector<float *> fft_pair_bf;   // the same as split BF16 fragments [nfp][14][64][16] (KIFMM_BF16X3)
    std::vector<float *> fft_pair_h;    // single FP16 fragments [nfp][14][64][8], scaled per frequency (KIFMM_M2L_FP16)
    std::vector<float *> fft_pair_b1;   // single BF16 fragments, the same layout and scaling (KIFMM_M2L_BF16)
    std::vector<float *> fft_pair_us;   // [nfp] the inverse of each frequency's fragment scale
    // near field in Fourier space (kifmm_ops_p2p_fft; leaves of 8^3): half spectra of the
    // kernel of the 27 neighbour offsets [27][1920] complex, per-leaf spectra of the sources
    // [nleaf][1920] complex, and the sums after the first inverse stage [nleaf][120][8]
    // complex (allocated when first enabled; the kernels write and read the 113 stored
    // columns of the 120, the others being conjugates)
    bool p2p_fft = false;
    float *near_gh = nullptr, *near_q = nullptr, *near_p = nullptr;
    float *spec_e = nullptr, *spec_p = nullptr;
    std::vector<float> m2l_scale;      // per level: max |M2L| (low precision storage divisor)
    int *taps = nullptr;               // all tap tables
    TapList t_single{}, t_m2m{}, t_l2l{}, t_m2l{}, t_p2p{}, t_m2l0{};
    // work buffers (sized for FP64)
    double *q = nullptr, *Sp = nullptr, *SpN = nullptr;   // leaf-ordered sources, far / near field
    std::vector<double *> cu, cd;
    float *amax = nullptr;
    int n_amax = 256;
    float *part = nullptr;             // tap-group partial sums of the M2L launches
    int64_t part_capacity = 0;         // floats
    // the near field runs on a second stream (then, with both Fourier forms, the coarse
    // levels' M2L down to level 4), joined by events; with the FFT form of M2L the finest
    // level's M2L runs on a third, beside the upward pass and the coarse levels, and level 3's
    // M2L on a fourth
    hipStream_t side = nullptr, fine = nullptr, coarse = nullptr;
    bool serial = false;             // kifmm_ops_serial: every pass on the calling stream, in order
    // P2M and L2P as MFMA fragments for the kernels fused with the permutes (FP32, leaves of
    // 8^3 cells): [KU / 32 tiles][64 chunks][64 lanes] and [16 tiles][KD / 8 chunks][64 lanes]
    float4 *p2m_frag = nullptr, *l2p_frag = nullptr;
    // the same in split BF16 (KIFMM_BF16X3): [KU / 32 tiles][32 chunks][hi, lo][64 lanes] and
    // [16 tiles][KD / 16 chunks, even][hi, lo][64 lanes] of 8 BF16 values
    uint4 *p2m_xf = nullptr, *l2p_xf = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, fork_fine = nullptr, join_fine = nullptr, join_coarse = nullptr;
    // per coarse level l (3 .. D - 1): c_u^l is ready (ev_up), its M2L is done (ev_m2l)
    std::vector<hipEvent_t> ev_up, ev_m2l;
    // per-pass timing (kifmm_profile_enable)
    bool prof = false;
    std::vector<hipEvent_t> ev;        // pool of events, recorded in pairs
    std::vector<int> ev_pass;          // pass of each recorded pair
    int ev_used = 0;
    double prof_ms[KIFMM_NPASS] = {};
    int64_t prof_calls[KIFMM_NPASS] = {};
};

// flags of the boxes at level l, or null when zero-source skipping is off
static const uint8_t *nz_of(kifmm_ops o, int l) {
    return o->skip_zero && l >= o->lmin && l < (int)o->nz.size() ? o->nz[l] : nullptr;
}

// wanted-target flags of the boxes at level l, or null when every target is wanted
static const uint8_t *want_of(kifmm_ops o, int l) {
    return l >= 0 && l < (int)o->want.size() ? o->want[l] : nullptr;
}

static void drain_profile(kifmm_ops o) {
    for (int i = 0; i < o->ev_used; ++i) {
        float ms = 0.f;
        (void)hipEventSynchronize(o->ev[2 * i + 1]);
        if (hipEventElapsedTime(&ms, o->ev[2 * i], o->ev[2 * i + 1]) == hipSuccess) {
            o->prof_ms[o->ev_pass[i]] += ms;
            o->prof_calls[o->ev_pass[i]] += 1;
        }
    }
    o->ev_used = 0;
}

static void clear_profile(kifmm_ops o) {
    for (hipEvent_t e : o->ev) (void)hipEventDestroy(e);
    o->ev.clear();
    o->ev_pass.clear();
    o->ev_used = 0;
    o->prof = false;
    for (int p = 0; p < KIFMM_NPASS; ++p) { o->prof_ms[p] = 0; o->prof_calls[p] = 0; }
}

// scoped event pair around one launch (no-op unless profiling is enabled and a
// free pair is left in the pool)
struct PassTimer {
    kifmm_ops o;
    int slot = -1;
    hipStream_t st;
    PassTimer(kifmm_ops ops, int pass, hipStream_t s) : o(ops), st(s) {
        if (pass < 0 || !o->prof || 2 * (o->ev_used + 1) > (int)o->ev.size()) return;
        slot = o->ev_used++;
        o->ev_pass[slot] = pass;
        (void)hipEventRecord(o->ev[2 * slot], st);
    }
    ~PassTimer() {
        if (slot >= 0) (void)hipEventRecord(o->ev[2 * slot + 1], st);
    }
};

// The near-field, finest-level and level-3 streams of the evaluations, one set per device,
// shared by every operator object and kept until the process ends.  HIP spreads streams over
// a few hardware queues (4 by default); a set per live object would put the passes of
// several objects, and the calling stream, on shared queues and serialise what should
// overlap.
static std::mutex g_stream_mu;
static std::vector<std::array<hipStream_t, 3>> g_streams;

static int shared_streams(hipStream_t *side, hipStream_t *fine, hipStream_t *coarse) {
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_stream_mu);
    if (dev >= (int)g_streams.size()) g_streams.resize(dev + 1, {nullptr, nullptr, nullptr});
    auto &p = g_streams[dev];
    for (hipStream_t &s : p)
        if (!s) KIFMM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *side = p[0];
    *fine = p[1];
    *coarse = p[2];
    return KIFMM_OK;
}

static void free_ops(kifmm_ops o) {
    if (!o) return;
    clear_profile(o);
    if (o->side) (void)hipStreamSynchronize(o->side);
    if (o->fine) (void)hipStreamSynchronize(o->fine);
    if (o->coarse) (void)hipStreamSynchronize(o->coarse);
    void *ptrs[] = {o->p2m32, o->m2m32, o->m2l32, o->l2l32, o->l2p32, o->p2p32, o->p2m64,
                    o->m2m64, o->m2l64, o->l2l64, o->l2p64, o->p2p64, o->m2lbf, o->m2lbf_lo,
                    o->p2mbf, o->m2mbf, o->l2lbf, o->l2pbf, o->p2mh, o->m2mh, o->l2lh, o->l2ph,
                    o->m2lh,  o->taps,  o->q,     o->Sp,    o->SpN,   o->amax,  o->part,
                    o->p2pbf, o->p2pbf_lo, o->amax_q, o->split_q, o->split_c, o->spec_e, o->spec_p,
                    o->p2m_frag, o->l2p_frag, o->p2m_xf, o->l2p_xf, o->m2l0_32, o->m2l0_64, o->lat_buf, o->lat_buf_c, o->spec_e_c, o->spec_p_c, o->near_gh, o->near_q, o->near_p};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (double *p : o->cu)
        if (p) (void)hipFree(p);
    for (uint8_t *p : o->nz)
        if (p) (void)hipFree(p);
    for (uint8_t *p : o->want)
        if (p) (void)hipFree(p);
    for (auto *v : {&o->fft_g, &o->lat_w, &o->lat_u, &o->fft_pair, &o->fft_pair_bf, &o->fft_pair_h, &o->fft_pair_b1,
                    &o->fft_pair_us})
        for (float *p : *v)
            if (p) (void)hipFree(p);
    for (double *p : o->cd)
        if (p) (void)hipFree(p);
    if (o->fork) (void)hipEventDestroy(o->fork);
    if (o->join) (void)hipEventDestroy(o->join);
    if (o->fork_fine) (void)hipEventDestroy(o->fork_fine);
    if (o->join_fine) (void)hipEventDestroy(o->join_fine);
    if (o->join_coarse) (void)hipEventDestroy(o->join_coarse);
    for (auto *v : {&o->ev_up, &o->ev_m2l})
        for (hipEvent_t e : *v)
            if (e) (void)hipEventDestroy(e);
    delete o;
}

// ------------------------------------------------------------------ checks --
static int check_grid(const kifmm_grid *g) {
    if (!g) return fail(KIFMM_EINVAL, "grid is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(KIFMM_EINVAL, "grid sizes must be > 0");
    if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0)) return fail(KIFMM_EINVAL, "cell sizes must be > 0");
    if (!std::isfinite(g->hx) || !std::isfinite(g->hy) || !std::isfinite(g->hz))
        return fail(KIFMM_EINVAL, "cell sizes must be finite");
    return KIFMM_OK;
}
static int check_kernel(const kifmm_kernel *k) {
    if (!k) return fail(KIFMM_EINVAL, "kernel is NULL");
    if (!(k->chi_min > 0) || !(k->chi_max > k->chi_min) || !std::isfinite(k->chi_max))
        return fail(KIFMM_EINVAL, "need 0 < chi_min < chi_max");
    if (!(k->p_o2 > 0) || !std::isfinite(k->p_o2)) return fail(KIFMM_EINVAL, "p_o2 must be > 0");
    return KIFMM_OK;
}

extern "C" {

const char *kifmm_last_error(void) { return g_err.c_str(); }

int direct_eval(const kifmm_grid *grid, const kifmm_kernel *kernel, const float *I_dev,
                double prefactor, const int64_t *tgt_idx_dev, int64_t n_tgt, double *out_dev,
                int32_t fp64_accumulate, void *stream) {
    KIFMM_TRY(check_grid(grid));
    KIFMM_TRY(check_kernel(kernel));
    if (n_tgt < 0) return fail(KIFMM_EINVAL, "n_tgt must be >= 0");
    if (n_tgt == 0) return KIFMM_OK;
    if (!I_dev || (!out_dev && n_tgt > 0)) return fail(KIFMM_EINVAL, "I_dev and out_dev must be non-NULL");
    const int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
    if (!tgt_idx_dev && n_tgt != N) return fail(KIFMM_EINVAL, "tgt_idx_dev NULL requires n_tgt == N");
    if (!std::isfinite(prefactor)) return fail(KIFMM_EINVAL, "prefactor must be finite");
    const char *ib = (const char *)I_dev, *ob = (const char *)out_dev;
    if (n_tgt > 0 && ob < ib + N * sizeof(float) && ib < ob + n_tgt * sizeof(double))
        return fail(KIFMM_EINVAL, "I_dev and out_dev overlap");
    return launch_direct(grid, kernel, I_dev, prefactor, tgt_idx_dev, n_tgt, out_dev,
                         fp64_accumulate ? 1 : 0, (hipStream_t)stream);
}

int kifmm_build_tree(const kifmm_grid *grid, int32_t max_leaf, void *stream, kifmm_tree *out) {
    if (!out) return fail(KIFMM_EINVAL, "out is NULL");
    KIFMM_TRY(check_grid(grid));
    if (max_leaf < 1) return fail(KIFMM_EINVAL, "max_leaf must be >= 1");
    if (grid->nx != grid->ny)
        return fail(KIFMM_EUNSUPPORTED, "nx must equal ny (a cube, or a column of cubes along z)");
    if (grid->hx != grid->hy) return fail(KIFMM_EUNSUPPORTED, "hx must equal hy");
    const int n = grid->nx, nz = grid->nz;
    if (n & (n - 1)) return fail(KIFMM_EUNSUPPORTED, "n must be a power of two");
    if (n > 1024) return fail(KIFMM_EUNSUPPORTED, "n must be <= 1024");
    const bool cube = nz == n && grid->hz == grid->hx;
    // leaves: ell x ell x ellz cells, ell the largest power of two that fits max_leaf; on a
    // cube ellz = ell, else the power of two closest (in ratio) to ell hx / hz, so that the
    // leaves are nearly cubic in space
    auto ellz_for = [&](int e) {
        if (cube) return e;
        const double want = e * grid->hx / grid->hz;
        int ez = 1;
        while (ez * 2 <= nz && std::fabs(std::log2(ez * 2.0 / want)) < std::fabs(std::log2(ez / want))) ez *= 2;
        return ez;
    };
    int ell = 0;
    for (int e = 1; e <= n; e *= 2)
        if ((int64_t)e * e * ellz_for(e) <= max_leaf) ell = e;
    if (ell < 4)
        return fail(KIFMM_EUNSUPPORTED, "leaves must hold at least 4 x 4 cells across (n >= 4, max_leaf large enough)");
    const int ellz = ellz_for(ell), nb = n / ell;
    if (nz % ((int64_t)ellz * nb) != 0)
        return fail(KIFMM_EUNSUPPORTED, "nz must be a multiple of ellz * nx / ell (a column of whole cubes of leaves)");
    const int R = nz / (ellz * nb);
    if (R > 64) return fail(KIFMM_EUNSUPPORTED, "at most 64 root cubes along z");
    if ((int64_t)n * n * nz > INT32_MAX) return fail(KIFMM_EUNSUPPORTED, "at most 2^31 - 1 cells");
    kifmm_tree t = new (std::nothrow) kifmm_tree_s();
    if (!t) return fail(KIFMM_ENOMEM, "host allocation failed");
    t->magic = g_magic.fetch_add(1);
    t->n = n;
    t->nz = nz;
    t->ell = ell;
    t->ellz = ellz;
    t->nb = nb;
    t->R = R;
    t->depth = 0;
    while ((1 << t->depth) < t->nb) ++t->depth;
    t->s = ell * ell * ellz;
    t->N = (int64_t)n * n * nz;
    t->h = grid->hx;
    t->hz = grid->hz;
    t->x0 = grid->x0;
    t->y0 = grid->y0;
    t->z0 = grid->z0;
    t->perm = nullptr;
    int rc = dmalloc(&t->perm, (size_t)t->N);
    if (rc == KIFMM_OK) rc = launch_morton_scatter(*t, (hipStream_t)stream);
    if (rc == KIFMM_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    if (rc != KIFMM_OK) {
        if (t->perm) (void)hipFree(t->perm);
        delete t;
        return rc;
    }
    *out = t;
    return KIFMM_OK;
}

int kifmm_tree_info(kifmm_tree tree, int32_t *depth, int32_t *leaf_side) {
    if (!tree) return fail(KIFMM_EINVAL, "tree is NULL");
    if (depth) *depth = tree->depth;
    if (leaf_side) *leaf_side = tree->ell;
    return KIFMM_OK;
}

int kifmm_tree_shape(kifmm_tree tree, int32_t *leaf_xy, int32_t *leaf_z, int32_t *roots) {
    if (!tree) return fail(KIFMM_EINVAL, "tree is NULL");
    if (leaf_xy) *leaf_xy = tree->ell;
    if (leaf_z) *leaf_z = tree->ellz;
    if (roots) *roots = tree->R;
    return KIFMM_OK;
}

int kifmm_tree_permutation(kifmm_tree tree, int64_t *perm_dev, void *stream) {
    if (!tree || !perm_dev) return fail(KIFMM_EINVAL, "tree and perm_dev must be non-NULL");
    return launch_perm_i64(*tree, perm_dev, (hipStream_t)stream);
}

void kifmm_tree_destroy(kifmm_tree tree) {
    if (!tree) return;
    if (tree->perm) (void)hipFree(tree->perm);
    delete tree;
}

void kifmm_ops_destroy(kifmm_ops ops) { free_ops(ops); }

int kifmm_ops_rank(kifmm_ops ops, int32_t level, int32_t *k_up, int32_t *k_down) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    if (level < ops->lmin || level > ops->D) return fail(KIFMM_EINVAL, "level out of range");
    if (k_up) *k_up = ops->ku[level];
    if (k_down) *k_down = ops->kd[level];
    return KIFMM_OK;
}

}  // extern "C"

// --------------------------------------------------------------- precompute --
namespace {

struct DevBuf {  // scoped FP64 scratch for the precompute
    std::vector<void *> ptrs;
    ~DevBuf() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    int get(T **p, size_t count) {
        int rc = dmalloc(p, count);
        if (rc == KIFMM_OK && *p) ptrs.push_back(*p);
        return rc;
    }
};

template <typename T>
int upload(DevBuf &db, const std::vector<T> &h, T **d, hipStream_t st) {
    KIFMM_TRY(db.get(d, h.size()));
    KIFMM_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return KIFMM_OK;
}

// truncated SVDs of a batch of same-shape matrices G(X_b, Y_b) (m x n).
// Output per batch item: UT (k x m) and W = V S^-1 (n x k), FP64 device.  The one-sided
// Jacobi method orthogonalises the columns of the matrix it is given, so a wide G
// (m < n) is factored through its transpose: G^T = U' S V'^T gives U = V', V = U'.
struct Factor {
    double *UT = nullptr, *W = nullptr;
    int k = 0, m = 0, n = 0;
};

int batched_tsvd(DevBuf &db, const std::vector<const double *> &X, const std::vector<const double *> &Y,
                 int m, int n, const kifmm_kernel &kern, double h, double rcond,
                 std::vector<Factor> &out, hipStream_t st) {
    const int B = (int)X.size();
    const bool trans = m < n;
    const int mg = m, ng = n;   // shape of G
    if (trans) std::swap(m, n);   // from here on: the factored matrix, n columns of length m
    const int npad = n + (n & 1);
    double *A, *V;
    KIFMM_TRY(db.get(&A, (size_t)B * npad * m));
    KIFMM_TRY(db.get(&V, (size_t)B * npad * npad));
    std::vector<double> eye((size_t)npad * npad, 0.0);
    for (int i = 0; i < npad; ++i) eye[(size_t)i * npad + i] = 1.0;
    for (int b = 0; b < B; ++b) {
        KIFMM_HIP(hipMemsetAsync(A + (size_t)b * npad * m, 0, sizeof(double) * npad * m, st));
        // columns stored contiguously: G transposed, or for a wide G its rows (= G^T's columns)
        KIFMM_TRY(launch_kmat(X[b], mg, Y[b], ng, nullptr, nullptr, 1, trans ? 0 : 1, kern, h,
                              A + (size_t)b * npad * m, st));
        KIFMM_HIP(hipMemcpyAsync(V + (size_t)b * npad * npad, eye.data(), eye.size() * sizeof(double),
                                 hipMemcpyHostToDevice, st));
    }
    std::vector<int> md(B, m), nd(B, n);
    int *mdd, *ndd;
    KIFMM_TRY(upload(db, md, &mdd, st));
    KIFMM_TRY(upload(db, nd, &ndd, st));
    unsigned long long *offd;
    KIFMM_TRY(db.get(&offd, (size_t)B));
    // Column pairs are rotated while |a_p . a_q| > tol ||a_p|| ||a_q||.  The dot
    // products of m-long FP64 columns carry rounding of order sqrt(m) * 1e-16, so tol
    // sits above that floor; a last sweep whose worst pair is below 1e-10 is accepted.
    const double tol = 1e-12;
    std::vector<unsigned long long> zeros(B, 0), offh(B);
    bool converged = false;
    double worst = 0.0;
    for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
        KIFMM_HIP(hipMemcpyAsync(offd, zeros.data(), B * sizeof(unsigned long long),
                                 hipMemcpyHostToDevice, st));
        for (int r = 0; r < npad - 1; ++r)
            KIFMM_TRY(launch_jacobi_round(A, V, mdd, ndd, npad, m, npad, (int64_t)npad * m,
                                          (int64_t)npad * npad, B, r, tol, offd, st));
        KIFMM_HIP(hipMemcpyAsync(offh.data(), offd, B * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
        KIFMM_HIP(hipStreamSynchronize(st));
        converged = true;
        worst = 0.0;
        for (int b = 0; b < B; ++b) {
            double v;
            std::memcpy(&v, &offh[b], sizeof(double));
            worst = std::max(worst, v);
            if (v > tol) converged = false;
        }
    }
    if (!converged && !(worst < 1e-10))
        return fail(KIFMM_EHIP, "Jacobi SVD did not converge in 60 sweeps (worst pair " + std::to_string(worst) + ")");
    double *sig;
    KIFMM_TRY(db.get(&sig, (size_t)B * npad));
    KIFMM_TRY(launch_colnorm(A, mdd, ndd, m, (int64_t)npad * m, npad, B, sig, st));
    std::vector<double> sh((size_t)B * npad);
    KIFMM_HIP(hipMemcpyAsync(sh.data(), sig, sh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    KIFMM_HIP(hipStreamSynchronize(st));
    out.assign(B, Factor());
    for (int b = 0; b < B; ++b) {
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        const double *s = sh.data() + (size_t)b * npad;
        std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return s[i] > s[j]; });
        const double smax = s[order[0]];
        int k = 0;
        while (k < n && s[order[k]] > rcond * smax) ++k;
        if (k == 0) return fail(KIFMM_EINVAL, "kernel matrix is zero at this pressure/size");
        std::vector<double> sk(k);
        for (int i = 0; i < k; ++i) sk[i] = s[order[i]];
        order.resize(k);
        int *ordd;
        double *skd;
        KIFMM_TRY(upload(db, order, &ordd, st));
        KIFMM_TRY(upload(db, sk, &skd, st));
        Factor &f = out[b];
        f.k = k; f.m = mg; f.n = ng;
        KIFMM_TRY(db.get(&f.UT, (size_t)k * mg));
        KIFMM_TRY(db.get(&f.W, (size_t)ng * k));
        if (!trans) {
            KIFMM_TRY(launch_svd_gather(A + (size_t)b * npad * m, V + (size_t)b * npad * npad, m, npad,
                                        m, n, k, ordd, skd, f.UT, f.W, st));
            continue;
        }
        // G^T = U' S V'^T: the gather gives U'^T (k x ng) and V' S^-1 (mg x k);
        // G's U^T = V'^T = (V' S^-1 S)^T and W = V S^-1 = U' S^-1
        double *ut2, *w2;
        KIFMM_TRY(db.get(&ut2, (size_t)k * ng));
        KIFMM_TRY(db.get(&w2, (size_t)mg * k));
        KIFMM_TRY(launch_svd_gather(A + (size_t)b * npad * m, V + (size_t)b * npad * npad, m, npad,
                                    m, n, k, ordd, skd, ut2, w2, st));
        std::vector<double> hu((size_t)k * ng), hw((size_t)mg * k), UT((size_t)k * mg), W((size_t)ng * k);
        KIFMM_HIP(hipMemcpyAsync(hu.data(), ut2, hu.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        KIFMM_HIP(hipMemcpyAsync(hw.data(), w2, hw.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        KIFMM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < k; ++r) {
            for (int i = 0; i < mg; ++i) UT[(size_t)r * mg + i] = hw[(size_t)i * k + r] * sk[r];
            for (int i = 0; i < ng; ++i) W[(size_t)i * k + r] = hu[(size_t)r * ng + i] / sk[r];
        }
        KIFMM_HIP(hipMemcpyAsync(f.UT, UT.data(), UT.size() * sizeof(double), hipMemcpyHostToDevice, st));
        KIFMM_HIP(hipMemcpyAsync(f.W, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, st));
        KIFMM_HIP(hipStreamSynchronize(st));   // UT and W are host vectors of this iteration
    }
    return KIFMM_OK;
}

// batch of operators  UT (k1 x m, shared) . G(X + sx_b, Y + sy_b) (m x n) . W (n x k2, shared or null)
int fused_ops(DevBuf &db, const double *UT, int k1, const double *X, int m, const double *Y, int n,
              const double *W, int k2, const double *sx, const double *sy, int batch,
              const kifmm_kernel &kern, double h, double *out, hipStream_t st) {
    double *G, *T1;
    KIFMM_TRY(db.get(&G, (size_t)batch * m * n));
    KIFMM_TRY(launch_kmat(X, m, Y, n, sx, sy, batch, 0, kern, h, G, st));
    if (UT && W) {
        KIFMM_TRY(db.get(&T1, (size_t)batch * k1 * n));
        KIFMM_TRY(launch_gemm_f64(k1, n, m, UT, m, 0, G, n, (int64_t)m * n, T1, n, (int64_t)k1 * n,
                                  batch, st));
        KIFMM_TRY(launch_gemm_f64(k1, k2, n, T1, n, (int64_t)k1 * n, W, k2, 0, out, k2,
                                  (int64_t)k1 * k2, batch, st));
    } else if (UT) {
        KIFMM_TRY(launch_gemm_f64(k1, n, m, UT, m, 0, G, n, (int64_t)m * n, out, n, (int64_t)k1 * n,
                                  batch, st));
    } else {
        KIFMM_TRY(launch_gemm_f64(m, k2, n, G, n, (int64_t)m * n, W, k2, 0, out, k2, (int64_t)m * k2,
                                  batch, st));
    }
    return KIFMM_OK;
}

template <typename T>
int store(const double *src, int M, int K, int batch, T *dst, int Mp, int Kp, double scale,
          hipStream_t st) {
    return launch_cast_pad<T>(src, M, K, (int64_t)M * K, dst, Mp, Kp, (int64_t)Mp * Kp, batch, scale, st);
}

int store_both(const double *src, int M, int K, int batch, float *d32, double *d64, int Mp, int Kp,
               hipStream_t st) {
    KIFMM_TRY(store<float>(src, M, K, batch, d32, Mp, Kp, 1.0, st));
    KIFMM_TRY(store<double>(src, M, K, batch, d64, Mp, Kp, 1.0, st));
    return KIFMM_OK;
}

int max_abs_host(const double *d, size_t count, double *out, hipStream_t st) {
    std::vector<double> h(count);
    KIFMM_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(double), hipMemcpyDeviceToHost, st));
    KIFMM_HIP(hipStreamSynchronize(st));
    double m = 0;
    for (double v : h) m = std::max(m, std::fabs(v));
    *out = m;
    return KIFMM_OK;
}

// Half spectra of the near-range kernel for leaves of 8^3 cells: for each neighbour offset o
// (in leaves, o = 9 (ox+1) + 3 (oy+1) + oz+1), g_o(d) = G((d - 8 o) h) for cell differences
// d in [-7, 7]^3 (the self value at d - 8 o = 0), placed at d mod 15, transformed over the
// 15^3 cyclic grid in FP64 and stored at f = (ky * 8 + kz) * 16 + kx, kz <= 7 (120 columns
// (ky, kz) of 16 slots, the 16th zero).
int build_near_spectra(DevBuf &db, kifmm_ops o, double h, hipStream_t st) {
    const int nd = 15 * 15 * 15;
    std::vector<double> dp(3 * nd), shifts(3 * 27);
    for (int d = 0; d < nd; ++d) {   // points -d h: G(0, -d h + 8 o h) = g_o(d)
        dp[3 * d] = -(d / 225 - 7) * h;
        dp[3 * d + 1] = -((d / 15) % 15 - 7) * h;
        dp[3 * d + 2] = -(d % 15 - 7) * h;
    }
    for (int t = 0; t < 27; ++t) {
        shifts[3 * t] = 8.0 * (t / 9 - 1) * h;
        shifts[3 * t + 1] = 8.0 * ((t / 3) % 3 - 1) * h;
        shifts[3 * t + 2] = 8.0 * (t % 3 - 1) * h;
    }
    double *org, *dpd, *shd, *G;
    KIFMM_TRY(upload(db, std::vector<double>(3, 0.0), &org, st));
    KIFMM_TRY(upload(db, dp, &dpd, st));
    KIFMM_TRY(upload(db, shifts, &shd, st));
    KIFMM_TRY(db.get(&G, (size_t)27 * nd));
    KIFMM_TRY(launch_kmat(org, 1, dpd, nd, nullptr, shd, 27, 0, o->kern, h, G, st));
    std::vector<double> g((size_t)27 * nd);
    KIFMM_HIP(hipMemcpyAsync(g.data(), G, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    KIFMM_HIP(hipStreamSynchronize(st));
    // 15-point transforms: 15 values per axis hold the differences -7..7 without overlap
    constexpr int N = 15, NZ = 8, NSLOT = 120 * 16;
    std::vector<double> cs(N), sn(N);
    for (int m = 0; m < N; ++m) {
        cs[m] = std::cos(2.0 * M_PI * m / N);
        sn[m] = std::sin(2.0 * M_PI * m / N);
    }
    std::vector<float> out((size_t)27 * NSLOT * 2, 0.0f);   // slot kx = 15 of every column stays 0
    std::vector<double> a((size_t)N * N * N), zr((size_t)N * N * NZ), zi(zr.size()), yr(zr.size()), yi(zr.size());
    for (int t = 0; t < 27; ++t) {
        for (int d = 0; d < nd; ++d) {   // every point of the cyclic grid is one difference
            const int x = (d / 225 - 7 + N) % N, y = ((d / 15) % 15 - 7 + N) % N, z = (d % 15 - 7 + N) % N;
            a[(x * N + y) * N + z] = g[(size_t)t * nd + d];
        }
        for (int x = 0; x < N; ++x)   // z
            for (int y = 0; y < N; ++y)
                for (int kz = 0; kz < NZ; ++kz) {
                    double re = 0, im = 0;
                    for (int z = 0; z < N; ++z) {
                        const double v = a[(x * N + y) * N + z];
                        re += v * cs[(kz * z) % N];
                        im -= v * sn[(kz * z) % N];
                    }
                    zr[(x * N + y) * NZ + kz] = re;
                    zi[(x * N + y) * NZ + kz] = im;
                }
        for (int x = 0; x < N; ++x)   // y
            for (int ky = 0; ky < N; ++ky)
                for (int kz = 0; kz < NZ; ++kz) {
                    double re = 0, im = 0;
                    for (int y = 0; y < N; ++y) {
                        const double vr = zr[(x * N + y) * NZ + kz], vi = zi[(x * N + y) * NZ + kz];
                        const double c = cs[(ky * y) % N], sv = sn[(ky * y) % N];
                        re += vr * c + vi * sv;
                        im += vi * c - vr * sv;
                    }
                    yr[(x * N + ky) * NZ + kz] = re;
                    yi[(x * N + ky) * NZ + kz] = im;
                }
        for (int kx = 0; kx < N; ++kx)   // x
            for (int ky = 0; ky < N; ++ky)
                for (int kz = 0; kz < NZ; ++kz) {
                    double re = 0, im = 0;
                    for (int x = 0; x < N; ++x) {
                        const double vr = yr[(x * N + ky) * NZ + kz], vi = yi[(x * N + ky) * NZ + kz];
                        const double c = cs[(kx * x) % N], sv = sn[(kx * x) % N];
                        re += vr * c + vi * sv;
                        im += vi * c - vr * sv;
                    }
                    const size_t f = (size_t)(ky * NZ + kz) * 16 + kx;
                    out[((size_t)t * NSLOT + f) * 2] = (float)re;
                    out[((size_t)t * NSLOT + f) * 2 + 1] = (float)im;
                }
    }
    KIFMM_TRY(dmalloc(&o->near_gh, out.size()));
    KIFMM_HIP(hipMemcpyAsync(o->near_gh, out.data(), out.size() * sizeof(float), hipMemcpyHostToDevice, st));
    KIFMM_HIP(hipStreamSynchronize(st));   // out is a host vector
    return KIFMM_OK;
}

// FFT form of M2L for the lattice layout.  With y^u = x^d = the m0^3 lattice of spacing t
// around the box centre, G(x^d_i, y^u_j + 2 r o) = g_o(i - j) with g_o(d) = G(d t - 2 r o).
// On the cyclic grid of N = 2 m0 - 1 points per axis the differences i - j never wrap onto
// one another, so the M2L product is the inverse DFT of DFT(g_o) times DFT(density).  Per
// level: the spectra of g_o for the 316 offsets at the stored frequencies of the lattice
// transforms (kz = 1 .. m0 - 1 at (kx N + ky)(m0 - 1) + kz - 1, then one of each conjugate
// pair of the plane kz = 0; real and imaginary parts interleaved), with the MFMA operator
// fragments of the parent-pair form; the map from upward coefficients to the equivalent
// density on the lattice, W_u; and the map from check potentials on the lattice to
// downward coefficients, U_d^T.  The transforms between lattice values and spectra run
// separably on the device (the conjugate-symmetric half counted twice where kz > 0).
int build_fft_m2l(DevBuf &db, kifmm_ops o, double Lside, double h, const std::vector<int> &m2lo,
                  const std::vector<Factor> &fu, const std::vector<Factor> &fd, hipStream_t st) {
    const int m = o->opts.m0, N = 2 * m - 1, D = o->D, KU = o->KU, KD = o->KD;
    const int n316 = (int)m2lo.size() / 3;
    // stored frequencies: kz = 1 .. m - 1 in full, and one of each conjugate pair of the plane
    // kz = 0 (the device transforms read the other as the conjugate of its mirror)
    const int H = m - 1, B0 = N * N * H;
    const int nf = B0 + m + H * N, nfp = pad_to(nf, 16), mf = 2 * nfp;
    const int nd = N * N * N, nlat = m * m * m;
    o->nfp = nfp;
    o->mf = mf;
    o->lrow = pad_to(nlat, 32);
    const double twopi_n = 2.0 * M_PI / N;
    auto phase = [&](int f, int x, int y, int z) {   // exact integer phase, reduced mod N
        int kx, ky, kz;
        if (f < B0) {
            kz = f % H + 1;
            kx = f / H / N;
            ky = f / H % N;
        } else if (f < B0 + m) {
            kx = 0;
            ky = f - B0;
            kz = 0;
        } else {
            kx = (f - B0 - m) / N + 1;
            ky = (f - B0 - m) % N;
            kz = 0;
        }
        const int64_t ph = (int64_t)kx * x + (int64_t)ky * y + (int64_t)kz * z;
        return twopi_n * (double)(((ph % N) + N) % N);
    };
    std::vector<double> FD((size_t)nd * 2 * nf);
    for (int d = 0; d < nd; ++d) {   // difference d = (dx, dy, dz) in [-(m-1), m-1]^3, C order
        const int dx = d / (N * N) - (m - 1), dy = (d / N) % N - (m - 1), dz = d % N - (m - 1);
        for (int f = 0; f < nf; ++f) {
            const double a = phase(f, dx, dy, dz);
            FD[(size_t)d * 2 * nf + 2 * f] = std::cos(a);
            FD[(size_t)d * 2 * nf + 2 * f + 1] = -std::sin(a);
        }
    }
    double *FDd, *org, *Dp, *sh, *G, *tmp;
    KIFMM_TRY(upload(db, FD, &FDd, st));
    KIFMM_TRY(upload(db, std::vector<double>(3, 0.0), &org, st));
    KIFMM_TRY(db.get(&Dp, (size_t)3 * nd));
    KIFMM_TRY(db.get(&sh, (size_t)3 * n316));
    KIFMM_TRY(db.get(&G, (size_t)n316 * nd));
    KIFMM_TRY(db.get(&tmp, (size_t)std::max(n316, std::max(KU, KD)) * 2 * nf));
    o->fft_g.assign(D + 1, nullptr);
    o->lat_w.assign(D + 1, nullptr);
    o->lat_u.assign(D + 1, nullptr);
    o->fft_pair.assign(D + 1, nullptr);
    o->fft_pair_bf.assign(D + 1, nullptr);
    o->fft_pair_h.assign(D + 1, nullptr);
    o->fft_pair_b1.assign(D + 1, nullptr);
    o->fft_pair_us.assign(D + 1, nullptr);
    // offset -> index into the 316 offsets, for the parent-pair matrices
    std::vector<int> oidx(343, -1);
    for (int t = 0; t < n316; ++t)
        oidx[((m2lo[3 * t] + 3) * 7 + (m2lo[3 * t + 1] + 3)) * 7 + (m2lo[3 * t + 2] + 3)] = t;
    for (int l = 2; l <= D; ++l) {
        const double r = Lside / std::ldexp(1.0, l + 1), t = 2.0 * o->opts.lattice_radius * r / (m - 1);
        std::vector<double> dp(3 * nd), shifts(3 * n316);
        for (int d = 0; d < nd; ++d) {   // points -d t: G(0, -d t + 2 r o) = g_o(d)
            dp[3 * d] = -(d / (N * N) - (m - 1)) * t;
            dp[3 * d + 1] = -((d / N) % N - (m - 1)) * t;
            dp[3 * d + 2] = -(d % N - (m - 1)) * t;
        }
        for (int i = 0; i < 3 * n316; ++i) shifts[i] = 2.0 * r * m2lo[i];
        KIFMM_HIP(hipMemcpyAsync(Dp, dp.data(), dp.size() * sizeof(double), hipMemcpyHostToDevice, st));
        KIFMM_HIP(hipMemcpyAsync(sh, shifts.data(), shifts.size() * sizeof(double), hipMemcpyHostToDevice, st));
        KIFMM_TRY(launch_kmat(org, 1, Dp, nd, nullptr, sh, n316, 0, o->kern, h, G, st));
        KIFMM_TRY(launch_gemm_f64(n316, 2 * nf, nd, G, nd, 0, FDd, 2 * nf, 0, tmp, 2 * nf, 0, 1, st));
        KIFMM_TRY(dmalloc(&o->fft_g[l], (size_t)n316 * mf));
        KIFMM_TRY(store<float>(tmp, n316, 2 * nf, 1, o->fft_g[l], n316, mf, 1.0, st));
        if (l >= 3) {
            // Parent-pair form: per frequency the 16 x 432 real matrix taking the spectra of
            // the 8 children of each of the 27 neighbour parents (k = 16 d + 2 c_s + re/im) to
            // the 8 children of the target parent (row = 2 c_t + re/im), laid out as MFMA
            // fragments [f][source parent d][lane][4 k-steps]: k-step 4 d + s of lane l holds
            // (row l % 16, k = 4 (4 d + s) + l / 16), so a lane loads one parent's 4 in one go.
            std::vector<double> gh((size_t)n316 * 2 * nf);
            KIFMM_HIP(hipMemcpyAsync(gh.data(), tmp, gh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            KIFMM_HIP(hipStreamSynchronize(st));
            // entry (row, k) of frequency f's matrix; offset index t = -1 where the two children
            // are adjacent (no M2L term)
            auto offset_of = [&](int row, int k) {
                const int ct = row >> 1, d = k / 16, cs = (k / 2) % 8;
                const int ov[3] = {2 * (d / 9 - 1) + ((cs >> 2) & 1) - ((ct >> 2) & 1),
                                   2 * ((d / 3) % 3 - 1) + ((cs >> 1) & 1) - ((ct >> 1) & 1),
                                   2 * (d % 3 - 1) + (cs & 1) - (ct & 1)};
                return oidx[((ov[0] + 3) * 7 + (ov[1] + 3)) * 7 + (ov[2] + 3)];
            };
            auto entry = [&](int t, int f, int row, int k) {
                const double gr = gh[(size_t)t * 2 * nf + 2 * f], gi = gh[(size_t)t * 2 * nf + 2 * f + 1];
                return (row & 1) == 0 ? ((k & 1) == 0 ? gr : -gi) : ((k & 1) == 0 ? gi : gr);
            };
            std::vector<float> am((size_t)nfp * 108 * 64, 0.f);
            for (int ks = 0; ks < 108; ++ks)
                for (int ln = 0; ln < 64; ++ln) {
                    const int row = ln & 15, k = 4 * ks + (ln >> 4), t = offset_of(row, k);
                    if (t < 0) continue;
                    for (int f = 0; f < nf; ++f)   // [f][d = ks / 4][lane][ks % 4]
                        am[(((size_t)f * 27 + ks / 4) * 64 + ln) * 4 + ks % 4] = (float)entry(t, f, row, k);
                }
            KIFMM_TRY(dmalloc(&o->fft_pair[l], am.size()));
            KIFMM_HIP(hipMemcpyAsync(o->fft_pair[l], am.data(), am.size() * sizeof(float), hipMemcpyHostToDevice, st));
            KIFMM_HIP(hipStreamSynchronize(st));   // am is a host vector of this iteration
            // The same matrices split into BF16 high and low parts (v = hi + lo, both rounded
            // to nearest even) as fragments of v_mfma_f32_16x16x32_bf16, K padded to 448:
            // [f][k-step (14)][lane][hi 8, lo 8], lane l holding (row l % 16, k = 32 k-step +
            // 8 (l / 16) + 0..7), source parents in the k order with 13 and 26 swapped (the
            // last k-step is then zero and is not read).
            auto bf16_bits = [](float v) {
                uint32_t u;
                std::memcpy(&u, &v, 4);
                u += 0x7fffu + ((u >> 16) & 1u);
                return (uint16_t)(u >> 16);
            };
            auto bf16_value = [](uint16_t b) {
                const uint32_t u = (uint32_t)b << 16;
                float v;
                std::memcpy(&v, &u, 4);
                return v;
            };
            std::vector<uint16_t> ab((size_t)nfp * 14 * 64 * 16, 0);
            for (int ks = 0; ks < 14; ++ks)
                for (int ln = 0; ln < 64; ++ln)
                    for (int j = 0; j < 8; ++j) {
                        // position q = k / 16 holds source parent d = q with 13 and 26 swapped
                        const int row = ln & 15, k = 32 * ks + 8 * (ln >> 4) + j, q = k / 16;
                        if (q >= 27) continue;
                        const int kd = 16 * (q == 13 ? 26 : (q == 26 ? 13 : q)) + k % 16;
                        const int t = offset_of(row, kd);
                        if (t < 0) continue;
                        for (int f = 0; f < nf; ++f) {
                            const double v = entry(t, f, row, kd);
                            const uint16_t hi = bf16_bits((float)v), lo = bf16_bits((float)(v - (double)bf16_value(hi)));
                            const size_t at = (((size_t)f * 14 + ks) * 64 + ln) * 16 + j;
                            ab[at] = hi;
                            ab[at + 8] = lo;
                        }
                    }
            KIFMM_TRY(dmalloc(&o->fft_pair_bf[l], ab.size() / 2));   // counted in floats
            KIFMM_HIP(hipMemcpyAsync(o->fft_pair_bf[l], ab.data(), ab.size() * sizeof(uint16_t), hipMemcpyHostToDevice, st));
            KIFMM_HIP(hipStreamSynchronize(st));
            // Single-part FP16 and BF16 fragments, [f][k-step (14)][lane][8] in the k order of
            // the split form, each frequency's matrix scaled by 2^(14 - e) (e the exponent of its
            // largest magnitude, so the entries fit FP16's range); us[f] undoes the scale.
            std::vector<float> smax(nfp, 0.f), us(nfp, 1.f);
            for (int ks = 0; ks < 14; ++ks)
                for (int ln = 0; ln < 64; ++ln)
                    for (int j = 0; j < 8; ++j) {
                        const int row = ln & 15, k = 32 * ks + 8 * (ln >> 4) + j, q = k / 16;
                        if (q >= 27) continue;
                        const int kd = 16 * (q == 13 ? 26 : (q == 26 ? 13 : q)) + k % 16;
                        const int t = offset_of(row, kd);
                        if (t < 0) continue;
                        for (int f = 0; f < nf; ++f)
                            smax[f] = std::max(smax[f], (float)std::fabs(entry(t, f, row, kd)));
                    }
            std::vector<float> sc(nfp, 1.f);
            for (int f = 0; f < nf; ++f)
                if (smax[f] > 0.f) {
                    int ex = 0;
                    std::frexp(smax[f], &ex);
                    sc[f] = std::ldexp(1.f, 14 - ex);
                    us[f] = std::ldexp(1.f, ex - 14);
                }
            std::vector<_Float16> ah((size_t)nfp * 14 * 64 * 8, (_Float16)0.f);
            std::vector<uint16_t> a1((size_t)nfp * 14 * 64 * 8, 0);
            for (int ks = 0; ks < 14; ++ks)
                for (int ln = 0; ln < 64; ++ln)
                    for (int j = 0; j < 8; ++j) {
                        const int row = ln & 15, k = 32 * ks + 8 * (ln >> 4) + j, q = k / 16;
                        if (q >= 27) continue;
                        const int kd = 16 * (q == 13 ? 26 : (q == 26 ? 13 : q)) + k % 16;
                        const int t = offset_of(row, kd);
                        if (t < 0) continue;
                        for (int f = 0; f < nf; ++f) {
                            const float v = (float)entry(t, f, row, kd) * sc[f];
                            const size_t at = (((size_t)f * 14 + ks) * 64 + ln) * 8 + j;
                            ah[at] = (_Float16)v;
                            a1[at] = bf16_bits(v);
                        }
                    }
            KIFMM_TRY(dmalloc(&o->fft_pair_h[l], ah.size() / 2));
            KIFMM_TRY(dmalloc(&o->fft_pair_b1[l], a1.size() / 2));
            KIFMM_TRY(dmalloc(&o->fft_pair_us[l], us.size()));
            KIFMM_HIP(hipMemcpyAsync(o->fft_pair_h[l], ah.data(), ah.size() * sizeof(_Float16), hipMemcpyHostToDevice, st));
            KIFMM_HIP(hipMemcpyAsync(o->fft_pair_b1[l], a1.data(), a1.size() * sizeof(uint16_t), hipMemcpyHostToDevice, st));
            KIFMM_HIP(hipMemcpyAsync(o->fft_pair_us[l], us.data(), us.size() * sizeof(float), hipMemcpyHostToDevice, st));
            KIFMM_HIP(hipStreamSynchronize(st));
        }
        const Factor &u = fu[l - 2], &dn = fd[l - 2];
        KIFMM_TRY(dmalloc(&o->lat_w[l], (size_t)o->lrow * KU));
        KIFMM_TRY(store<float>(u.W, nlat, u.k, 1, o->lat_w[l], o->lrow, KU, 1.0, st));
        KIFMM_TRY(dmalloc(&o->lat_u[l], (size_t)KD * o->lrow));
        KIFMM_TRY(store<float>(dn.UT, dn.k, nlat, 1, o->lat_u[l], KD, o->lrow, 1.0, st));
        KIFMM_HIP(hipStreamSynchronize(st));   // dp and shifts are reused by the next level
    }
    const size_t nbx = (size_t)1 << (3 * D);
    KIFMM_TRY(dmalloc(&o->spec_e, nbx * mf));
    KIFMM_TRY(dmalloc(&o->spec_p, nbx * mf));
    KIFMM_TRY(dmalloc(&o->lat_buf, nbx * o->lrow));
    if (D >= 3) {
        const size_t ncoarse = (nbx / 8 * 8 - 64) / 7;   // boxes of levels 2 .. D - 1
        KIFMM_TRY(dmalloc(&o->spec_e_c, ncoarse * mf));
        KIFMM_TRY(dmalloc(&o->spec_p_c, ncoarse * mf));
        KIFMM_TRY(dmalloc(&o->lat_buf_c, ncoarse * o->lrow));
    }
    o->m2l_fft = true;
    return KIFMM_OK;
}

int build_ops(kifmm_tree tree, kifmm_ops o, hipStream_t st) {
    DevBuf db;
    const int D = o->D, s = o->s, ell = o->ell, ellz = o->ellz, R = o->R, lmin = o->lmin;
    const bool cube = R == 1 && ellz == ell && tree->hz == tree->h;
    // a root cube's sides (x = y, z): box half-widths at level l are these over 2^(l+1)
    const double h = tree->h, hz = tree->hz, Lside = tree->h * tree->n, Lz = hz * ellz * o->nb;
    const kifmm_kernel &kern = o->kern;
    auto rx_of = [&](int l) { return Lside / std::ldexp(1.0, l + 1); };
    auto rz_of = [&](int l) { return Lz / std::ldexp(1.0, l + 1); };
    o->ku.assign(D + 1, 0);
    o->kd.assign(D + 1, 0);

    // near-range matrices (27 taps) -- always needed
    std::vector<int> nbr;
    for (int x = -1; x <= 1; ++x)
        for (int y = -1; y <= 1; ++y)
            for (int z = -1; z <= 1; ++z) {
                nbr.push_back(x);
                nbr.push_back(y);
                nbr.push_back(z);
            }
    int *nbrd;
    KIFMM_TRY(upload(db, nbr, &nbrd, st));
    double *p2p;
    KIFMM_TRY(db.get(&p2p, (size_t)27 * s * s));
    KIFMM_TRY(launch_near(ell, ellz, h, hz, nbrd, 27, kern, p2p, st));
    KIFMM_TRY(dmalloc(&o->p2p32, (size_t)27 * s * s));
    KIFMM_TRY(dmalloc(&o->p2p64, (size_t)27 * s * s));
    KIFMM_TRY(store_both(p2p, s, s, 27, o->p2p32, o->p2p64, s, s, st));
    if (ell == 8 && cube) KIFMM_TRY(build_near_spectra(db, o, h, st));
    {
        double mx;
        KIFMM_TRY(max_abs_host(p2p, (size_t)27 * s * s, &mx, st));
        if (!(mx > 0)) mx = 1.0;
        o->p2p_scale = (float)mx;
        KIFMM_TRY(dmalloc(&o->p2pbf, (size_t)27 * s * s));
        KIFMM_TRY(dmalloc(&o->p2pbf_lo, (size_t)27 * s * s));
        KIFMM_TRY(store<__bf16>(p2p, s, s, 27, o->p2pbf, s, s, 1.0 / mx, st));
        KIFMM_TRY(launch_cast_pad_lo(p2p, s, s, (int64_t)s * s, o->p2pbf_lo, s, s, (int64_t)s * s, 27,
                                     1.0 / mx, st));
    }

    // tap tables
    std::vector<int> taps;
    auto add_list = [&](TapList &tl, int nclass, int ntaps, const std::vector<int> &op,
                        const std::vector<int> &off) {
        tl.nclass = nclass;
        tl.ntaps = ntaps;
        tl.op_dev = (int *)(size_t)taps.size();  // offset, fixed up after upload
        taps.insert(taps.end(), op.begin(), op.end());
        tl.off_dev = (int *)(size_t)taps.size();
        taps.insert(taps.end(), off.begin(), off.end());
    };
    {
        std::vector<int> op(27), off(27);
        for (int t = 0; t < 27; ++t) {
            op[t] = t;
            off[t] = pack_off(nbr[3 * t], nbr[3 * t + 1], nbr[3 * t + 2]);
        }
        add_list(o->t_p2p, 1, 27, op, off);
        add_list(o->t_single, 1, 1, {0}, {0});
        std::vector<int> c8(8);
        std::iota(c8.begin(), c8.end(), 0);
        add_list(o->t_m2m, 1, 8, c8, c8);
        add_list(o->t_l2l, 8, 1, c8, std::vector<int>(8, 0));
    }
    const std::vector<int> m2lo = m2l_offsets();
    const int n316 = (int)m2lo.size() / 3;
    {
        std::vector<int> op, off;
        int ntaps = -1;
        for (int p = 0; p < 8; ++p) {
            const int par[3] = {(p >> 2) & 1, (p >> 1) & 1, p & 1};
            int cnt = 0;
            for (int t = 0; t < n316; ++t) {
                bool ok = true;
                for (int a = 0; a < 3; ++a) {
                    const int f = floordiv2(par[a] + m2lo[3 * t + a]);
                    if (f < -1 || f > 1) ok = false;
                }
                if (!ok) continue;
                op.push_back(t);
                off.push_back(pack_off(m2lo[3 * t], m2lo[3 * t + 1], m2lo[3 * t + 2]));
                ++cnt;
            }
            if (ntaps < 0) ntaps = cnt;
            if (cnt != ntaps) return fail(KIFMM_EINVAL, "internal: uneven interaction lists");
        }
        add_list(o->t_m2l, 8, ntaps, op, off);
    }
    if (R > 2) {   // level 0 of a column of cubes: every root two or more apart
        std::vector<int> op, off;
        for (int dz = -(R - 1); dz <= R - 1; ++dz) {
            if (std::abs(dz) < 2) continue;
            op.push_back((int)op.size());
            off.push_back(pack_off(0, 0, dz));
        }
        o->n0 = (int)op.size();
        add_list(o->t_m2l0, 1, o->n0, op, off);
    }
    KIFMM_TRY(dmalloc(&o->taps, taps.size()));
    KIFMM_HIP(hipMemcpyAsync(o->taps, taps.data(), taps.size() * sizeof(int), hipMemcpyHostToDevice, st));
    for (TapList *tl : {&o->t_p2p, &o->t_single, &o->t_m2m, &o->t_l2l, &o->t_m2l, &o->t_m2l0}) {
        if (tl->ntaps == 0) continue;
        tl->op_dev = o->taps + (size_t)tl->op_dev;
        tl->off_dev = o->taps + (size_t)tl->off_dev;
    }

    // work buffers
    KIFMM_TRY(dmalloc(&o->q, (size_t)tree->N));
    KIFMM_TRY(dmalloc(&o->Sp, (size_t)tree->N));
    KIFMM_TRY(dmalloc(&o->SpN, (size_t)tree->N));
    KIFMM_TRY(shared_streams(&o->side, &o->fine, &o->coarse));
    KIFMM_HIP(hipEventCreateWithFlags(&o->fork, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&o->join, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&o->fork_fine, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&o->join_fine, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&o->join_coarse, hipEventDisableTiming));
    KIFMM_TRY(dmalloc(&o->amax, (size_t)o->n_amax));
    KIFMM_TRY(dmalloc(&o->amax_q, (size_t)o->n_amax));
    o->cu.assign(D + 1, nullptr);
    o->cd.assign(D + 1, nullptr);
    o->ev_up.assign(D + 1, nullptr);
    o->ev_m2l.assign(D + 1, nullptr);
    for (int l = 3; l < D && cube; ++l) {
        KIFMM_HIP(hipEventCreateWithFlags(&o->ev_up[l], hipEventDisableTiming));
        KIFMM_HIP(hipEventCreateWithFlags(&o->ev_m2l[l], hipEventDisableTiming));
    }
    if (D < lmin) {
        KIFMM_HIP(hipStreamSynchronize(st));
        return KIFMM_OK;
    }

    // point sets per level, relative to the box centre
    std::vector<PointSets> ps(D + 1);
    std::vector<double *> yu(D + 1), xu(D + 1), yd(D + 1), xd(D + 1);
    for (int l = lmin; l <= D; ++l) {
        // the unit point sets, stretched to the box (half-widths rx, rx, rz)
        ps[l] = make_point_sets(o->opts, 1.0);
        const double sc[3] = {rx_of(l), rx_of(l), rz_of(l)};
        for (auto *v : {&ps[l].yu, &ps[l].xu, &ps[l].yd, &ps[l].xd})
            for (size_t i = 0; i < v->size(); ++i) (*v)[i] *= sc[i % 3];
        KIFMM_TRY(upload(db, ps[l].yu, &yu[l], st));
        KIFMM_TRY(upload(db, ps[l].xu, &xu[l], st));
        KIFMM_TRY(upload(db, ps[l].yd, &yd[l], st));
        KIFMM_TRY(upload(db, ps[l].xd, &xd[l], st));
    }
    const int nyu = (int)ps[lmin].yu.size() / 3, nxu = (int)ps[lmin].xu.size() / 3;
    const int nyd = (int)ps[lmin].yd.size() / 3, nxd = (int)ps[lmin].xd.size() / 3;

    // truncated SVDs of the check-to-equivalent matrices, every level
    std::vector<const double *> X, Y;
    for (int l = lmin; l <= D; ++l) { X.push_back(xu[l]); Y.push_back(yu[l]); }
    std::vector<Factor> fu, fd;
    KIFMM_TRY(batched_tsvd(db, X, Y, nxu, nyu, kern, h, o->opts.rcond, fu, st));
    X.clear(); Y.clear();
    for (int l = lmin; l <= D; ++l) { X.push_back(xd[l]); Y.push_back(yd[l]); }
    KIFMM_TRY(batched_tsvd(db, X, Y, nxd, nyd, kern, h, o->opts.rcond, fd, st));
    int kumax = 0, kdmax = 0;
    for (int l = lmin; l <= D; ++l) {
        o->ku[l] = fu[l - lmin].k;
        o->kd[l] = fd[l - lmin].k;
        kumax = std::max(kumax, o->ku[l]);
        kdmax = std::max(kdmax, o->kd[l]);
    }
    const int KU = pad_to(kumax, 32), KD = pad_to(kdmax, 32);
    o->KU = KU;
    o->KD = KD;
    auto UTu = [&](int l) { return fu[l - lmin].UT; };
    auto Wu = [&](int l) { return fu[l - lmin].W; };
    auto UTd = [&](int l) { return fd[l - lmin].UT; };
    auto Wd = [&](int l) { return fd[l - lmin].W; };

    // leaf cell centres relative to the leaf centre, C order
    std::vector<double> P;
    for (int i = 0; i < ell; ++i)
        for (int j = 0; j < ell; ++j)
            for (int k = 0; k < ellz; ++k) {
                P.push_back((i + 0.5) * h - 0.5 * ell * h);
                P.push_back((j + 0.5) * h - 0.5 * ell * h);
                P.push_back((k + 0.5) * hz - 0.5 * ellz * hz);
            }
    double *Pd;
    KIFMM_TRY(upload(db, P, &Pd, st));

    // P2M (eq. (s2m)): U_u^T G(x^u, leaf cells)       k_u x s
    {
        double *tmp;
        KIFMM_TRY(db.get(&tmp, (size_t)o->ku[D] * s));
        KIFMM_TRY(fused_ops(db, UTu(D), o->ku[D], xu[D], nxu, Pd, s, nullptr, 0, nullptr, nullptr, 1,
                            kern, h, tmp, st));
        KIFMM_TRY(dmalloc(&o->p2m32, (size_t)KU * s));
        KIFMM_TRY(dmalloc(&o->p2m64, (size_t)KU * s));
        KIFMM_TRY(store_both(tmp, o->ku[D], s, 1, o->p2m32, o->p2m64, KU, s, st));
    }
    // L2P: G(leaf cells, y^d) V_d S^-1                  s x k_d
    {
        double *tmp;
        KIFMM_TRY(db.get(&tmp, (size_t)s * o->kd[D]));
        KIFMM_TRY(fused_ops(db, nullptr, 0, Pd, s, yd[D], nyd, Wd(D), o->kd[D], nullptr, nullptr, 1,
                            kern, h, tmp, st));
        KIFMM_TRY(dmalloc(&o->l2p32, (size_t)s * KD));
        KIFMM_TRY(dmalloc(&o->l2p64, (size_t)s * KD));
        KIFMM_TRY(store_both(tmp, s, o->kd[D], 1, o->l2p32, o->l2p64, s, KD, st));
    }
    // their MFMA fragments for the kernels fused with the permutes
    if (leafgemm_fits(*tree, KU, KD)) {
        KIFMM_TRY(dmalloc(&o->p2m_frag, (size_t)KU * s / 4));
        const int l2p_chunks = l2p_fragment_chunks(KD);   // KD / 8 rounded up to even
        KIFMM_TRY(dmalloc(&o->l2p_frag, (size_t)(s / 32) * l2p_chunks * 64));
        KIFMM_TRY(launch_pack_fragments(o->p2m32, KU, s, s, s / 8, o->p2m_frag, st));
        KIFMM_TRY(launch_pack_fragments(o->l2p32, s, KD, KD, l2p_chunks, o->l2p_frag, st));
        const int l2p_chunks_x3 = l2p_fragment_chunks_x3(KD);   // KD / 16 rounded up to even
        KIFMM_TRY(dmalloc(&o->p2m_xf, (size_t)(KU / 32) * (s / 16) * 128));
        KIFMM_TRY(dmalloc(&o->l2p_xf, (size_t)(s / 32) * l2p_chunks_x3 * 128));
        KIFMM_TRY(launch_pack_fragments_x3(o->p2m64, KU, s, s, s / 16, o->p2m_xf, st));
        KIFMM_TRY(launch_pack_fragments_x3(o->l2p64, s, KD, KD, l2p_chunks_x3, o->l2p_xf, st));
    }
    // child centre offsets at a level of half-widths (r, r, rz): (2c - 1) r per axis
    auto child_shifts = [&](double r, double rz) {
        std::vector<double> v;
        for (int c = 0; c < 8; ++c) {
            v.push_back((2 * ((c >> 2) & 1) - 1) * r);
            v.push_back((2 * ((c >> 1) & 1) - 1) * r);
            v.push_back((2 * (c & 1) - 1) * rz);
        }
        return v;
    };
    // M2M (eq. (m2m)), levels lmin..D-1 (block l - lmin): U_u^T(l) G(x^u(l), y^u(l+1) + child) W_u(l+1)
    if (D > lmin) {
        KIFMM_TRY(dmalloc(&o->m2m32, (size_t)(D - lmin) * 8 * KU * KU));
        KIFMM_TRY(dmalloc(&o->m2m64, (size_t)(D - lmin) * 8 * KU * KU));
        KIFMM_TRY(dmalloc(&o->l2l32, (size_t)(D - lmin) * 8 * KD * KD));
        KIFMM_TRY(dmalloc(&o->l2l64, (size_t)(D - lmin) * 8 * KD * KD));
        for (int l = lmin; l <= D - 1; ++l) {
            double *sh, *tmp;
            KIFMM_TRY(upload(db, child_shifts(rx_of(l + 1), rz_of(l + 1)), &sh, st));
            KIFMM_TRY(db.get(&tmp, (size_t)8 * o->ku[l] * o->ku[l + 1]));
            KIFMM_TRY(fused_ops(db, UTu(l), o->ku[l], xu[l], nxu, yu[l + 1], nyu, Wu(l + 1),
                                o->ku[l + 1], nullptr, sh, 8, kern, h, tmp, st));
            const size_t so = (size_t)(l - lmin) * 8 * KU * KU;
            KIFMM_TRY(store_both(tmp, o->ku[l], o->ku[l + 1], 8, o->m2m32 + so, o->m2m64 + so, KU, KU, st));
        }
        // L2L (eq. (l2l)), levels lmin+1..D (block l - lmin - 1): U_d^T(l) G(x^d(l) + child, y^d(l-1)) W_d(l-1)
        for (int l = lmin + 1; l <= D; ++l) {
            double *sh, *tmp;
            KIFMM_TRY(upload(db, child_shifts(rx_of(l), rz_of(l)), &sh, st));
            KIFMM_TRY(db.get(&tmp, (size_t)8 * o->kd[l] * o->kd[l - 1]));
            KIFMM_TRY(fused_ops(db, UTd(l), o->kd[l], xd[l], nxd, yd[l - 1], nyd, Wd(l - 1),
                                o->kd[l - 1], sh, nullptr, 8, kern, h, tmp, st));
            const size_t so = (size_t)(l - lmin - 1) * 8 * KD * KD;
            KIFMM_TRY(store_both(tmp, o->kd[l], o->kd[l - 1], 8, o->l2l32 + so, o->l2l64 + so, KD, KD, st));
        }
    }
    // M2L (eq. (m2l)), levels lmin..D (block l - lmin; level 0 of a column of cubes has its
    // own list), 316 offsets: U_d^T G(x^d, y^u + 2 r o) W_u
    {
        const size_t per = (size_t)n316 * KD * KU;
        const size_t nlev = (size_t)(D - lmin + 1);
        KIFMM_TRY(dmalloc(&o->m2l32, nlev * per));
        KIFMM_TRY(dmalloc(&o->m2l64, nlev * per));
        KIFMM_TRY(dmalloc(&o->m2lbf, nlev * per));
        KIFMM_TRY(dmalloc(&o->m2lbf_lo, nlev * per));
        KIFMM_TRY(dmalloc(&o->m2lh, nlev * per));
        o->m2l_scale.assign(D + 1, 1.0f);
        double *G, *T1, *tmp, *sh;
        const size_t maxk = (size_t)std::max(kumax, kdmax);
        KIFMM_TRY(db.get(&G, (size_t)n316 * nxd * nyu));
        KIFMM_TRY(db.get(&T1, (size_t)n316 * maxk * nyu));
        KIFMM_TRY(db.get(&tmp, (size_t)n316 * maxk * maxk));
        KIFMM_TRY(db.get(&sh, (size_t)3 * n316));
        for (int l = std::max(lmin, 1); l <= D; ++l) {
            std::vector<double> shifts(3 * n316);
            for (int i = 0; i < 3 * n316; ++i) shifts[i] = 2.0 * (i % 3 == 2 ? rz_of(l) : rx_of(l)) * m2lo[i];
            KIFMM_HIP(hipMemcpyAsync(sh, shifts.data(), shifts.size() * sizeof(double),
                                     hipMemcpyHostToDevice, st));
            const int kd = o->kd[l], ku = o->ku[l];
            KIFMM_TRY(launch_kmat(xd[l], nxd, yu[l], nyu, nullptr, sh, n316, 0, kern, h, G, st));
            KIFMM_TRY(launch_gemm_f64(kd, nyu, nxd, UTd(l), nxd, 0, G, nyu, (int64_t)nxd * nyu, T1,
                                      nyu, (int64_t)kd * nyu, n316, st));
            KIFMM_TRY(launch_gemm_f64(kd, ku, nyu, T1, nyu, (int64_t)kd * nyu, Wu(l), ku, 0, tmp, ku,
                                      (int64_t)kd * ku, n316, st));
            const size_t so = (size_t)(l - lmin) * per;
            KIFMM_TRY(store_both(tmp, kd, ku, n316, o->m2l32 + so, o->m2l64 + so, KD, KU, st));
            double mx;
            KIFMM_TRY(max_abs_host(tmp, (size_t)n316 * kd * ku, &mx, st));
            if (!(mx > 0)) mx = 1.0;
            o->m2l_scale[l] = (float)mx;
            KIFMM_TRY(store<__bf16>(tmp, kd, ku, n316, o->m2lbf + so, KD, KU, 1.0 / mx, st));
            KIFMM_TRY(launch_cast_pad_lo(tmp, kd, ku, (int64_t)kd * ku, o->m2lbf_lo + so, KD, KU,
                                         (int64_t)KD * KU, n316, 1.0 / mx, st));
            KIFMM_TRY(store<_Float16>(tmp, kd, ku, n316, o->m2lh + so, KD, KU, 1.0 / mx, st));
        }
        if (o->n0 > 0) {   // level 0 of a column of cubes: roots (0, 0, dz) apart, |dz| >= 2
            std::vector<double> shifts;
            for (int dz = -(R - 1); dz <= R - 1; ++dz)
                if (std::abs(dz) >= 2) {
                    shifts.push_back(0.0);
                    shifts.push_back(0.0);
                    shifts.push_back(2.0 * rz_of(0) * dz);
                }
            const int n0 = o->n0, kd = o->kd[0], ku = o->ku[0];
            KIFMM_HIP(hipMemcpyAsync(sh, shifts.data(), shifts.size() * sizeof(double), hipMemcpyHostToDevice, st));
            KIFMM_TRY(launch_kmat(xd[0], nxd, yu[0], nyu, nullptr, sh, n0, 0, kern, h, G, st));
            KIFMM_TRY(launch_gemm_f64(kd, nyu, nxd, UTd(0), nxd, 0, G, nyu, (int64_t)nxd * nyu, T1,
                                      nyu, (int64_t)kd * nyu, n0, st));
            KIFMM_TRY(launch_gemm_f64(kd, ku, nyu, T1, nyu, (int64_t)kd * nyu, Wu(0), ku, 0, tmp, ku,
                                      (int64_t)kd * ku, n0, st));
            KIFMM_TRY(dmalloc(&o->m2l0_32, (size_t)n0 * KD * KU));
            KIFMM_TRY(dmalloc(&o->m2l0_64, (size_t)n0 * KD * KU));
            KIFMM_TRY(store_both(tmp, kd, ku, n0, o->m2l0_32, o->m2l0_64, KD, KU, st));
        }
    }
    // BF16 and FP16 copies of the surface operators, each divided by its maximum magnitude
    {
        auto lowp = [&](const double *src, int M, int K, int batch, __bf16 **bf, _Float16 **hh, float *scale) {
            double mx;
            KIFMM_TRY(max_abs_host(src, (size_t)M * K * batch, &mx, st));
            if (!(mx > 0)) mx = 1.0;
            *scale = (float)mx;
            KIFMM_TRY(dmalloc(bf, (size_t)M * K * batch));
            KIFMM_TRY(dmalloc(hh, (size_t)M * K * batch));
            KIFMM_TRY(store<__bf16>(src, M, K, batch, *bf, M, K, 1.0 / mx, st));
            return store<_Float16>(src, M, K, batch, *hh, M, K, 1.0 / mx, st);
        };
        KIFMM_TRY(lowp(o->p2m64, KU, s, 1, &o->p2mbf, &o->p2mh, &o->p2m_scale));
        KIFMM_TRY(lowp(o->l2p64, s, KD, 1, &o->l2pbf, &o->l2ph, &o->l2p_scale));
        o->m2m_scale.assign(D + 1, 1.0f);
        o->l2l_scale.assign(D + 1, 1.0f);
        if (D > lmin) {
            KIFMM_TRY(dmalloc(&o->m2mbf, (size_t)(D - lmin) * 8 * KU * KU));
            KIFMM_TRY(dmalloc(&o->m2mh, (size_t)(D - lmin) * 8 * KU * KU));
            KIFMM_TRY(dmalloc(&o->l2lbf, (size_t)(D - lmin) * 8 * KD * KD));
            KIFMM_TRY(dmalloc(&o->l2lh, (size_t)(D - lmin) * 8 * KD * KD));
        }
        for (int l = lmin; l <= D - 1; ++l) {   // M2M into level l: block l - lmin
            const size_t so = (size_t)(l - lmin) * 8 * KU * KU;
            double mx;
            KIFMM_TRY(max_abs_host(o->m2m64 + so, (size_t)8 * KU * KU, &mx, st));
            if (!(mx > 0)) mx = 1.0;
            o->m2m_scale[l] = (float)mx;
            KIFMM_TRY(store<__bf16>(o->m2m64 + so, KU, KU, 8, o->m2mbf + so, KU, KU, 1.0 / mx, st));
            KIFMM_TRY(store<_Float16>(o->m2m64 + so, KU, KU, 8, o->m2mh + so, KU, KU, 1.0 / mx, st));
        }
        for (int l = lmin + 1; l <= D; ++l) {   // L2L into level l: block l - lmin - 1
            const size_t so = (size_t)(l - lmin - 1) * 8 * KD * KD;
            double mx;
            KIFMM_TRY(max_abs_host(o->l2l64 + so, (size_t)8 * KD * KD, &mx, st));
            if (!(mx > 0)) mx = 1.0;
            o->l2l_scale[l] = (float)mx;
            KIFMM_TRY(store<__bf16>(o->l2l64 + so, KD, KD, 8, o->l2lbf + so, KD, KD, 1.0 / mx, st));
            KIFMM_TRY(store<_Float16>(o->l2l64 + so, KD, KD, 8, o->l2lh + so, KD, KD, 1.0 / mx, st));
        }
    }
    if (o->opts.layout == KIFMM_LAYOUT_LATTICE && cube) KIFMM_TRY(build_fft_m2l(db, o, Lside, h, m2lo, fu, fd, st));
    for (int l = lmin; l <= D; ++l) {
        const size_t nbx = (size_t)R << (3 * l);
        KIFMM_TRY(dmalloc(&o->cu[l], nbx * KU));
        KIFMM_TRY(dmalloc(&o->cd[l], nbx * KD));
    }
    o->split_c_n = ((int64_t)R << (3 * D)) * KU;
    KIFMM_TRY(dmalloc(&o->split_c, (size_t)(2 * o->split_c_n)));
    o->split_q_n = tree->N;
    KIFMM_TRY(dmalloc(&o->split_q, (size_t)(2 * o->split_q_n)));
    // scratch for the tap-group split of the M2L launches: up to 64 M floats
    // (the launcher uses fewer groups when a split would not fit)
    int64_t need = 0;
    for (int l = lmin; l <= D; ++l) {
        const int64_t nbx = (int64_t)R << (3 * l);
        const int64_t base = std::max<int64_t>(1, ((nbx / 8 + 63) / 64) * ((KD + 127) / 128) * 8);
        int64_t g = std::min<int64_t>(o->t_m2l.ntaps, (2048 + base - 1) / base);
        need = std::max(need, g * nbx * KD);
    }
    o->part_capacity = std::min<int64_t>(need, (int64_t)64 << 20);
    KIFMM_TRY(dmalloc(&o->part, (size_t)o->part_capacity));
    KIFMM_HIP(hipStreamSynchronize(st));
    return KIFMM_OK;
}

// ------------------------------------------------------------- evaluation --
template <typename TA, typename TI, typename TO>
TapArgs<TA, TI, TO> tap(const TA *A, int64_t a_stride, int M, int K, const TI *in, int64_t in_ld, TO *out,
                        int64_t out_ld, int mode, int nl, const TapList &tl, int cls_stride,
                        int64_t n_per_class, int accumulate, int zroots = 1) {
    TapArgs<TA, TI, TO> p{};
    p.A = A; p.A2 = nullptr; p.a_stride = a_stride; p.M = M; p.K = K;
    p.in = in; p.in2 = nullptr; p.in_ld = in_ld; p.out = out; p.out_ld = out_ld;
    p.mode = mode; p.nl = nl; p.zroots = zroots; p.nclass = tl.nclass; p.cls_stride = cls_stride;
    p.n_per_class = n_per_class; p.n_boxes = n_per_class * tl.nclass;
    p.tap_op = tl.op_dev; p.tap_off = tl.off_dev; p.ntaps = tl.ntaps;
    p.accumulate = accumulate;
    p.part = nullptr; p.part_capacity = 0; p.groups = 1;
    p.amax = nullptr; p.n_amax = 0; p.op_scale = 1.0f;
    p.pass = PASS_GENERIC;
    return p;
}

int run(const TapArgs<float, float, float> &p, hipStream_t st) { return run_tap_f32(p, st); }

int run(const TapArgs<double, double, double> &p, hipStream_t st) { return run_tap_f64(p, st); }

// A surface-operator pass (P2M, M2M, L2L, L2P) with BF16 or FP16 operands (KIFMM_BF16,
// KIFMM_FP16): the input is divided by its maximum magnitude (device-side partial maxima) and
// rounded while it is staged, the operator was stored divided by its own maximum, and the
// products accumulate in FP32.
template <typename TL>
int lowp_pass(kifmm_ops o, const TL *A, int64_t a_stride, int M, int K, const float *in, int64_t n_in, int64_t in_ld,
              float *out, int64_t out_ld, int mode, const TapList &tl, int nclass, int64_t nper, int acc, float scale,
              const uint8_t *in_nz, const uint8_t *out_need, bool split, hipStream_t st) {
    KIFMM_TRY(run_amax(in, n_in, o->amax, o->n_amax, st));
    auto p = tap<TL, float>(A, a_stride, M, K, in, in_ld, out, out_ld, mode, 0, tl, nclass, nper, acc);
    p.amax = o->amax;
    p.n_amax = o->n_amax;
    p.op_scale = scale;
    p.in_nz = in_nz;
    p.out_need = out_need;
    if (split) {
        p.part = o->part;
        p.part_capacity = o->part_capacity;
    }
    return run_tap_lp<TL>(p, false, st);
}

template <typename T>
struct OpSet {
    const T *p2m, *m2m, *m2l, *l2l, *l2p, *p2p;
};

// Precisions whose M2L runs in the FFT form when it is on: FP32, the split-BF16 modes, and
// the single-part M2L modes (their parent-pair products in FP16 or BF16)
static bool fft_precision(int precision) {
    return precision == KIFMM_FP32 || precision == KIFMM_BF16X3 || precision == KIFMM_M2L_BF16X3 ||
           precision == KIFMM_M2L_FP16 || precision == KIFMM_M2L_BF16;
}

// M2L of one level (eq. (m2l)) into cd[l], in the requested arithmetic
template <typename T>
int m2l_level(kifmm_ops o, const OpSet<T> &ops, int l, int precision, int acc, hipStream_t st) {
    const int KU = o->KU, KD = o->KD;
    const int64_t nper = (int64_t)o->R << (3 * (l - 1));   // boxes per parity class
    const size_t per = (size_t)316 * KD * KU;
    const size_t so = (size_t)(l - o->lmin) * per;
    const int zr = o->R;
    if (l == 0) {   // a column of cubes: the roots two or more apart (FP32 or FP64 operators)
        if (o->n0 == 0) return KIFMM_OK;
        const T *A0 = sizeof(T) == 8 ? (const T *)o->m2l0_64 : (const T *)o->m2l0_32;
        auto p = tap<T, T>(A0, (int64_t)KD * KU, KD, KU, (T *)o->cu[0], KU, (T *)o->cd[0], KD, SRC_NBR, 1,
                           o->t_m2l0, 1, o->R, acc, zr);
        p.in_nz = nz_of(o, 0);
        p.out_need = want_of(o, 0);
        p.pass = PASS_M2L;
        return run(p, st);
    }
    if constexpr (sizeof(T) == 4) {
        if (o->m2l_fft && fft_precision(precision)) {
            // FFT form: equivalent densities on the lattice, their spectra, pointwise
            // products, check potentials on the lattice, coefficients
            const int64_t nbx = (int64_t)1 << (3 * l);
            const int lr = o->lrow;
            const bool fine = l == o->D;   // the coarser levels have buffers of their own
            const size_t off = fine ? 0 : (((size_t)1 << (3 * l)) - 64) / 7;   // boxes of levels 2 .. l - 1
            float *lat = fine ? o->lat_buf : o->lat_buf_c + off * lr, *se = fine ? o->spec_e : o->spec_e_c + off * o->mf,
                  *sp = fine ? o->spec_p : o->spec_p_c + off * o->mf;
            auto pf = tap<float, float>(o->lat_w[l], 0, lr, KU, (const float *)o->cu[l], KU, lat, lr, SRC_SAME, 0,
                                        o->t_single, 1, nbx, 0);
            pf.in_nz = nz_of(o, l);
            KIFMM_TRY(run(pf, st));
            KIFMM_TRY(run_m2l_lattice(0, o->opts.m0, lat, nbx, o->nfp, lr, nz_of(o, l), se, st));
            if (o->fft_pair[l] && (precision == KIFMM_BF16X3 || precision == KIFMM_M2L_BF16X3))
                KIFMM_TRY(run_m2l_pair_bf16x3(se, o->fft_pair_bf[l], 1 << l, o->nfp, want_of(o, l), nz_of(o, l), sp, st));
            else if (o->fft_pair[l] && (precision == KIFMM_M2L_FP16 || precision == KIFMM_M2L_BF16)) {
                const bool h = precision == KIFMM_M2L_FP16;
                KIFMM_TRY(run_m2l_pair_lp1(h ? 1 : 0, se, h ? o->fft_pair_h[l] : o->fft_pair_b1[l], o->fft_pair_us[l],
                                           1 << l, o->nfp, want_of(o, l), nz_of(o, l), sp, st));
            }
            else if (o->fft_pair[l])
                KIFMM_TRY(run_m2l_pair_mfma(se, o->fft_pair[l], 1 << l, o->nfp, want_of(o, l), nz_of(o, l), sp, st));
            else
                KIFMM_TRY(run_m2l_hadamard(se, o->fft_g[l], o->t_m2l.op_dev, o->t_m2l.off_dev, o->t_m2l.ntaps, 1 << l,
                                           o->nfp, want_of(o, l), nz_of(o, l), sp, st));
            KIFMM_TRY(run_m2l_lattice(1, o->opts.m0, sp, nbx, o->nfp, lr, want_of(o, l), lat, st));
            auto pi = tap<float, float>(o->lat_u[l], 0, KD, lr, (const float *)lat, lr, (float *)o->cd[l],
                                        KD, SRC_SAME, 0, o->t_single, 1, nbx, acc);
            pi.out_need = want_of(o, l);
            pi.pass = PASS_M2L;
            return run(pi, st);
        }
        if (precision == KIFMM_M2L_BF16 || precision == KIFMM_M2L_FP16 || precision == KIFMM_M2L_BF16X3 ||
            precision == KIFMM_BF16X3 || precision == KIFMM_BF16 || precision == KIFMM_FP16) {
            const bool fp16 = precision == KIFMM_M2L_FP16 || precision == KIFMM_FP16;
            const int64_t ncu = ((int64_t)o->R << (3 * l)) * KU;
            KIFMM_TRY(run_amax((const float *)o->cu[l], ncu, o->amax, o->n_amax, st));
            const int64_t ldA = (int64_t)KD * KU;
            const bool x3 = precision == KIFMM_M2L_BF16X3 || precision == KIFMM_BF16X3;
            if (KD > 64) {   // staged kernel on the split coefficients
                if (fp16) {
                    _Float16 *hi = (_Float16 *)o->split_c;
                    KIFMM_TRY(run_split_lp<_Float16>((const float *)o->cu[l], ncu, o->amax, o->n_amax, hi, nullptr, st));
                    auto p = tap<_Float16, _Float16>(o->m2lh + so, ldA, KD, KU, hi, KU, (float *)o->cd[l], KD, SRC_NBR,
                                                     1 << l, o->t_m2l, 8, nper, acc, zr);
                    p.amax = o->amax; p.n_amax = o->n_amax; p.op_scale = o->m2l_scale[l];
                    p.part = o->part; p.part_capacity = o->part_capacity;
                    p.in_nz = nz_of(o, l);
                    p.out_need = want_of(o, l);
                    p.pass = PASS_M2L;
                    return run_tap_lp_staged<_Float16>(p, false, st);
                }
                __bf16 *hi = (__bf16 *)o->split_c, *lo = hi + o->split_c_n;
                KIFMM_TRY(run_split_lp<__bf16>((const float *)o->cu[l], ncu, o->amax, o->n_amax, hi, x3 ? lo : nullptr, st));
                auto p = tap<__bf16, __bf16>(o->m2lbf + so, ldA, KD, KU, hi, KU, (float *)o->cd[l], KD, SRC_NBR, 1 << l,
                                             o->t_m2l, 8, nper, acc, zr);
                p.A2 = o->m2lbf_lo + so;
                p.in2 = lo;
                p.amax = o->amax; p.n_amax = o->n_amax; p.op_scale = o->m2l_scale[l];
                p.part = o->part; p.part_capacity = o->part_capacity;
                p.in_nz = nz_of(o, l);
                p.out_need = want_of(o, l);
                p.pass = PASS_M2L;
                return run_tap_lp_staged<__bf16>(p, x3, st);
            }
            if (fp16) {
                auto p = tap<_Float16, float>(o->m2lh + so, ldA, KD, KU, (float *)o->cu[l], KU,
                                              (float *)o->cd[l], KD, SRC_NBR, 1 << l, o->t_m2l, 8, nper, acc, zr);
                p.amax = o->amax; p.n_amax = o->n_amax; p.op_scale = o->m2l_scale[l];
                p.part = o->part; p.part_capacity = o->part_capacity;
                p.in_nz = nz_of(o, l);
                p.out_need = want_of(o, l);
                p.pass = PASS_M2L;
                return run_tap_lp<_Float16>(p, false, st);
            }
            auto p = tap<__bf16, float>(o->m2lbf + so, ldA, KD, KU, (float *)o->cu[l], KU,
                                        (float *)o->cd[l], KD, SRC_NBR, 1 << l, o->t_m2l, 8, nper, acc, zr);
            p.A2 = o->m2lbf_lo + so;
            p.amax = o->amax; p.n_amax = o->n_amax; p.op_scale = o->m2l_scale[l];
            p.part = o->part; p.part_capacity = o->part_capacity;
            p.in_nz = nz_of(o, l);
            p.out_need = want_of(o, l);
            p.pass = PASS_M2L;
            return run_tap_lp<__bf16>(p, x3, st);
        }
    }
    auto p = tap<T, T>(ops.m2l + so, (int64_t)KD * KU, KD, KU, (T *)o->cu[l], KU, (T *)o->cd[l], KD, SRC_NBR,
                       1 << l, o->t_m2l, 8, nper, acc, zr);
    if constexpr (sizeof(T) == 4) {
        p.part = o->part;
        p.part_capacity = o->part_capacity;
    }
    p.in_nz = nz_of(o, l);
    p.out_need = want_of(o, l);
    p.pass = PASS_M2L;
    return run(p, st);
}

// near field (eq. (nearfar), direct part, with the self cell) of every leaf into out
// I_grid (FP32, Fourier form only): the sources read from the grid-order input times vol
// instead of q
template <typename T>
int p2p_pass(kifmm_ops o, const OpSet<T> &ops, const T *q, T *out, int precision, hipStream_t st,
             const float *I_grid = nullptr, float vol = 1.f) {
    const int s = o->s, nb = o->nb;
    const int64_t nleaf = (int64_t)o->R * nb * nb * nb;
    if constexpr (sizeof(T) == 4) {
        if (o->p2p_fft && nb >= 4) {   // FP32 arithmetic in every single-precision mode
            for (int stage = 0; stage < 3; ++stage) {
                PassTimer pt(o, stage == 1 ? KIFMM_PASS_NEAR_PRODUCTS : -1, st);
                KIFMM_TRY(run_near_fft_stage(stage, (const float *)q, o->near_gh, nb, want_of(o, o->D), nz_of(o, o->D),
                                             o->near_q, o->near_p, (float *)out, st, I_grid, vol));
            }
            return KIFMM_OK;
        }
        if (precision == KIFMM_BF16X3) {
            KIFMM_TRY(run_amax((const float *)q, nleaf * s, o->amax_q, o->n_amax, st));
            if (s > 64) {   // staged kernel on the split sources
                __bf16 *hi = (__bf16 *)o->split_q, *lo = hi + o->split_q_n;
                KIFMM_TRY(run_split_lp<__bf16>((const float *)q, nleaf * s, o->amax_q, o->n_amax, hi, lo, st));
                auto p = tap<__bf16, __bf16>(o->p2pbf, (int64_t)s * s, s, s, hi, s, (float *)out, s, SRC_NBR, nb,
                                             o->t_p2p, 1, nleaf, 0, o->R);
                p.A2 = o->p2pbf_lo;
                p.in2 = lo;
                p.amax = o->amax_q; p.n_amax = o->n_amax; p.op_scale = o->p2p_scale;
                p.in_nz = nz_of(o, o->D);
                p.out_need = want_of(o, o->D);
                p.pass = PASS_P2P;
                return run_tap_lp_staged<__bf16>(p, true, st);
            }
            auto p = tap<__bf16, float>(o->p2pbf, (int64_t)s * s, s, s, (const float *)q, s, (float *)out, s,
                                        SRC_NBR, nb, o->t_p2p, 1, nleaf, 0, o->R);
            p.A2 = o->p2pbf_lo;
            p.amax = o->amax_q; p.n_amax = o->n_amax; p.op_scale = o->p2p_scale;
            p.in_nz = nz_of(o, o->D);
            p.out_need = want_of(o, o->D);
            p.pass = PASS_P2P;
            return run_tap_lp<__bf16>(p, true, st);
        }
    }
    auto p = tap<T, T>(ops.p2p, (int64_t)s * s, s, s, q, s, out, s, SRC_NBR, nb, o->t_p2p, 1, nleaf, 0, o->R);
    p.in_nz = nz_of(o, o->D);
    p.out_need = want_of(o, o->D);
    p.pass = PASS_P2P;
    return run(p, st);
}

// Schedule (Section 3, algorithm outline):
//   stream st : permute in -> [fork] -> P2M -> M2M (l = D-1..2) -> for l = 2..D:
//               L2L (l > 2) then M2L -> L2P -> [wait join] -> permute out (far + near)
//   side      : [wait fork] -> P2P with the self cell -> [join]
// nz[leaf] = 1 if any of the leaf's s sources is nonzero (one wave per leaf)
template <typename T>
__global__ void leaf_nonzero_kernel(const T *__restrict__ q, int64_t nleaf, int s, uint8_t *__restrict__ nz) {
    const int lane = threadIdx.x & 63;
    for (int64_t L = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; L < nleaf;
         L += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        bool any = false;
        for (int i = lane; i < s; i += 64) any |= q[L * s + i] != (T)0;
        const uint64_t m = __ballot(any);
        if (lane == 0) nz[L] = m != 0;
    }
}

// parent[b] = OR of the 8 children 8b .. 8b+7 (Morton order)
__global__ void parent_nonzero_kernel(const uint8_t *__restrict__ child, int64_t nparent, uint8_t *__restrict__ parent) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nparent; b += (int64_t)gridDim.x * blockDim.x) {
        uint8_t v = 0;
        for (int c = 0; c < 8; ++c) v |= child[8 * b + c];
        parent[b] = v != 0;
    }
}

template <typename T>
int mark_nonzero_sources(kifmm_ops o, const T *q, hipStream_t st) {
    const int64_t nleaf = (int64_t)o->R * o->nb * o->nb * o->nb;
    int64_t blocks = (nleaf * 64 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(leaf_nonzero_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, q, nleaf, o->s, o->nz[o->D]);
    KIFMM_HIP(hipGetLastError());
    for (int l = o->D - 1; l >= o->lmin; --l) {
        const int64_t n = (int64_t)o->R << (3 * l);
        hipLaunchKernelGGL(parent_nonzero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, o->nz[l + 1], n,
                           o->nz[l]);
        KIFMM_HIP(hipGetLastError());
    }
    return KIFMM_OK;
}

// Error path of an evaluation whose side streams were forked: the streams are joined back
// into the calling stream before the error is returned, so that no later work on the calling
// stream (the next evaluation's permute into q, a caller's read of S) overlaps kernels still
// running on them, and a stream capture stays joined.
struct ForkJoin {
    kifmm_ops o;
    hipStream_t st, side, fine, coarse;
    bool side_forked = false, fine_forked = false, coarse_forked = false;
    ~ForkJoin() {
        if (side_forked && side != st) {
            (void)hipEventRecord(o->join, side);
            (void)hipStreamWaitEvent(st, o->join, 0);
        }
        if (fine_forked && fine != st) {
            (void)hipEventRecord(o->join_fine, fine);
            (void)hipStreamWaitEvent(st, o->join_fine, 0);
        }
        if (coarse_forked && coarse != st) {
            (void)hipEventRecord(o->join_coarse, coarse);
            (void)hipStreamWaitEvent(st, o->join_coarse, 0);
        }
    }
};

template <typename T>
int eval_typed(kifmm_tree t, kifmm_ops o, const T *I, T *S, double prefactor, int precision,
               hipStream_t st) {
    OpSet<T> ops;
    if constexpr (sizeof(T) == 8) ops = {o->p2m64, o->m2m64, o->m2l64, o->l2l64, o->l2p64, o->p2p64};
    else ops = {o->p2m32, o->m2m32, o->m2l32, o->l2l32, o->l2p32, o->p2p32};
    T *q = (T *)o->q, *Sp = (T *)o->Sp, *SpN = (T *)o->SpN;
    const int D = o->D, s = o->s, nb = o->nb, KU = o->KU, KD = o->KD, R = o->R, lmin = o->lmin;
    const int64_t nleaf = (int64_t)R * nb * nb * nb;
    // the cell volume goes in with the sources (q = I h^3), the prefactor on the way out:
    // FP32 sums of G I alone reach 1e37 for fine cells and bright sources
    const T vol = (T)(t->h * t->h * t->hz), scale = (T)prefactor;
    // every translation GEMM with BF16 or FP16 operands
    const bool lowp = sizeof(T) == 4 && (precision == KIFMM_BF16 || precision == KIFMM_FP16);
    // P2M fused with the way into leaf order, L2P with the sum and the way out (FP32 GEMMs,
    // leaves of 8^3 cells); with zero-source flags P2M keeps the tap GEMM, which skips them
    const bool fused_in = sizeof(T) == 4 && D >= 2 && o->p2m_frag && !lowp && !o->skip_zero &&
                          (uintptr_t)I % 16 == 0;
    const bool fused_out = sizeof(T) == 4 && D >= 2 && o->l2p_frag && !lowp && (uintptr_t)S % 16 == 0;
    // the side streams, or the calling stream itself when every pass is to run in order
    // (kifmm_ops_serial: per-kernel timings without overlap)
    hipStream_t side = o->serial ? st : o->side, fine = o->serial ? st : o->fine;
    hipStream_t coarse = o->serial ? st : o->coarse;
    ForkJoin fj{o, st, side, fine, coarse};
    // With the fused way in and the near field in Fourier space, the near field reads the
    // grid-order input itself (no leaf-ordered copy of the sources is written): its stream is
    // forked before P2M, which then runs beside the near field's first transform.
    const bool near_grid = fused_in && o->p2p_fft && nb >= 4 && D >= lmin;
    if (near_grid) {
        KIFMM_HIP(hipEventRecord(o->fork, st));
        KIFMM_HIP(hipStreamWaitEvent(side, o->fork, 0));
        fj.side_forked = true;
        {
            PassTimer pt(o, KIFMM_PASS_P2P, side);
            KIFMM_TRY(p2p_pass<T>(o, ops, nullptr, SpN, precision, side, (const float *)I, (float)vol));
        }
        KIFMM_HIP(hipEventRecord(o->join, side));
    }
    if (fused_in) {
        PassTimer pt(o, KIFMM_PASS_P2M, st);
        if (precision == KIFMM_BF16X3)
            KIFMM_TRY(run_p2m_permute_in_x3(*t, (const float *)I, (float)vol, o->p2m_xf, KU,
                                            near_grid ? nullptr : (float *)q, (float *)o->cu[D], st));
        else
            KIFMM_TRY(run_p2m_permute_in(*t, (const float *)I, (float)vol, o->p2m_frag, KU,
                                         near_grid ? nullptr : (float *)q, (float *)o->cu[D], st));
    } else {
        PassTimer pt(o, KIFMM_PASS_PERMUTE_IN, st);
        KIFMM_TRY(launch_permute_in<T>(*t, I, vol, q, st));
    }
    if (o->skip_zero && D >= lmin) KIFMM_TRY(mark_nonzero_sources<T>(o, q, st));
    if (D < lmin) {   // one cube of at most 2^3 leaves: every leaf is in every other leaf's near range
        {
            PassTimer pt(o, KIFMM_PASS_P2P, st);
            KIFMM_TRY(p2p_pass<T>(o, ops, q, Sp, precision, st));
        }
        PassTimer pt(o, KIFMM_PASS_PERMUTE_OUT, st);
        return launch_permute_out<T>(*t, Sp, scale, want_of(o, D), S, st);
    }
    // near field on the side stream, forked as early as possible: whatever runs beside it
    // waits for its long workgroups (forking it later, after the upward pass or before the
    // finest M2L level, measured slower)
    if (!near_grid) {
        KIFMM_HIP(hipEventRecord(o->fork, st));
        KIFMM_HIP(hipStreamWaitEvent(side, o->fork, 0));
        fj.side_forked = true;
        {
            PassTimer pt(o, KIFMM_PASS_P2P, side);
            KIFMM_TRY(p2p_pass<T>(o, ops, q, SpN, precision, side));
        }
        KIFMM_HIP(hipEventRecord(o->join, side));
    }
    // far field: upward pass, downward pass, local expansion at the cells
    if (!fused_in) {
        PassTimer pt(o, KIFMM_PASS_P2M, st);
        if (lowp) {
            if (precision == KIFMM_BF16)
                KIFMM_TRY(lowp_pass<__bf16>(o, o->p2mbf, 0, KU, s, (const float *)q, nleaf * s, s, (float *)o->cu[D], KU,
                                            SRC_SAME, o->t_single, 1, nleaf, 0, o->p2m_scale, nz_of(o, D), nullptr, false, st));
            else
                KIFMM_TRY(lowp_pass<_Float16>(o, o->p2mh, 0, KU, s, (const float *)q, nleaf * s, s, (float *)o->cu[D], KU,
                                              SRC_SAME, o->t_single, 1, nleaf, 0, o->p2m_scale, nz_of(o, D), nullptr, false, st));
        } else {
            auto p = tap<T, T>(ops.p2m, 0, KU, s, q, s, (T *)o->cu[D], KU, SRC_SAME, 0, o->t_single, 1, nleaf, 0);
            p.in_nz = nz_of(o, D);
            KIFMM_TRY(run(p, st));
        }
    }
    // FFT form of M2L: the finest level's M2L needs only the leaves' coefficients, so it runs
    // on its own stream beside the upward pass and the coarse levels (their latency-bound
    // small launches leave most of the chip to it), into cd[D]; the L2L into level D then
    // adds to it.  The coarse levels use spectra buffers of their own.
    const bool fine_apart = sizeof(T) == 4 && D >= 3 && o->m2l_fft && fft_precision(precision);
    if (fine_apart) {
        KIFMM_HIP(hipEventRecord(o->fork_fine, st));
        KIFMM_HIP(hipStreamWaitEvent(fine, o->fork_fine, 0));
        fj.fine_forked = true;
        {
            PassTimer pt(o, KIFMM_PASS_M2L, fine);
            KIFMM_TRY(m2l_level<T>(o, ops, D, precision, 0, fine));
        }
        KIFMM_HIP(hipEventRecord(o->join_fine, fine));
    }
    // With the near field in Fourier space its stream is free early: the M2L of levels
    // D - 1 .. 4 then runs there, each as soon as M2M has made that level's coefficients,
    // into cd[l], and level 3's on a stream of its own; the main stream does level 2 and the
    // L2L chain, each L2L adding to the M2L sum (the coarse chain of small launches is
    // otherwise the step's longest path).
    const bool coarse_side = fine_apart && D >= 4 && o->p2p_fft && nb >= 4;
    for (int l = D - 1; l >= lmin; --l) {
        const int64_t nbl = (int64_t)R << (3 * l);   // boxes of level l
        if (lowp) {
            const size_t so = (size_t)(l - lmin) * 8 * KU * KU;
            const int64_t nin = 8 * nbl * KU;
            PassTimer pt(o, KIFMM_PASS_M2M, st);
            if (precision == KIFMM_BF16)
                KIFMM_TRY(lowp_pass<__bf16>(o, o->m2mbf + so, (int64_t)KU * KU, KU, KU, (const float *)o->cu[l + 1], nin,
                                            KU, (float *)o->cu[l], KU, SRC_CHILD, o->t_m2m, 1, nbl, 0,
                                            o->m2m_scale[l], nz_of(o, l + 1), nullptr, true, st));
            else
                KIFMM_TRY(lowp_pass<_Float16>(o, o->m2mh + so, (int64_t)KU * KU, KU, KU, (const float *)o->cu[l + 1], nin,
                                              KU, (float *)o->cu[l], KU, SRC_CHILD, o->t_m2m, 1, nbl, 0,
                                              o->m2m_scale[l], nz_of(o, l + 1), nullptr, true, st));
        } else {
            const T *A = ops.m2m + (size_t)(l - lmin) * 8 * KU * KU;
            PassTimer pt(o, KIFMM_PASS_M2M, st);
            auto p = tap<T, T>(A, (int64_t)KU * KU, KU, KU, (T *)o->cu[l + 1], KU, (T *)o->cu[l], KU, SRC_CHILD, 0,
                               o->t_m2m, 1, nbl, 0);
            p.in_nz = nz_of(o, l + 1);
            if constexpr (sizeof(T) == 4) {
                p.part = o->part;
                p.part_capacity = o->part_capacity;
            }
            KIFMM_TRY(run(p, st));
        }
        if (coarse_side && l >= 3) KIFMM_HIP(hipEventRecord(o->ev_up[l], st));
    }
    if (coarse_side) {   // the events waited for below are all recorded (enqueued) above
        // finest first: level D - 1 is the longest and its coefficients are ready first (the
        // coarsest-first order, which lets the L2L chain start earlier, measured 20 us slower
        // per step as a graph).  Level 3 runs beside them on its own stream, as soon as its
        // coefficients exist (behind level 4 on the near-field stream it ended the step's
        // longest chain; level 4 on its own stream instead measured the same, every coarse
        // level on one stream of its own or each on its own slower)
        for (int l = D - 1; l >= 3; --l) {
            hipStream_t ls = l == 3 ? coarse : side;
            if (l == 3) fj.coarse_forked = true;
            KIFMM_HIP(hipStreamWaitEvent(ls, o->ev_up[l], 0));
            {
                PassTimer pt(o, KIFMM_PASS_M2L, ls);
                KIFMM_TRY(m2l_level<T>(o, ops, l, precision, 0, ls));
            }
            KIFMM_HIP(hipEventRecord(o->ev_m2l[l], ls));
        }
        KIFMM_HIP(hipEventRecord(o->join, side));
    }
    for (int l = lmin; l <= D; ++l) {
        // cd[l] holds the M2L sum already: the finest level (own stream), the coarse levels
        // 3 .. D - 1 (near-field stream)
        const bool m2l_done = (fine_apart && l == D) || (coarse_side && l >= 3);
        const int64_t npar = (int64_t)R << (3 * (l - 1));   // boxes of level l - 1 (l > lmin)
        if (l > lmin) {
            // the finest level's M2L (own stream) and the coarse ones (near-field stream) have
            // written cd[l]; the L2L adds to it.  (Issuing the finest L2L first and letting the
            // finest M2L's last map add to it measured no faster as a graph, slower eagerly.)
            if (fine_apart && l == D) KIFMM_HIP(hipStreamWaitEvent(st, o->join_fine, 0));
            else if (m2l_done) {
                KIFMM_HIP(hipStreamWaitEvent(st, o->ev_m2l[l], 0));
                if (l == 3) fj.coarse_forked = false;   // level 3's stream joined
            }
            PassTimer pt(o, KIFMM_PASS_L2L, st);
            if (lowp) {
                const size_t so = (size_t)(l - lmin - 1) * 8 * KD * KD;
                const int64_t nin = npar * KD, nper = npar;
                if (precision == KIFMM_BF16)
                    KIFMM_TRY(lowp_pass<__bf16>(o, o->l2lbf + so, (int64_t)KD * KD, KD, KD, (const float *)o->cd[l - 1], nin,
                                                KD, (float *)o->cd[l], KD, SRC_PARENT, o->t_l2l, 8, nper, m2l_done ? 1 : 0,
                                                o->l2l_scale[l], nullptr, want_of(o, l), false, st));
                else
                    KIFMM_TRY(lowp_pass<_Float16>(o, o->l2lh + so, (int64_t)KD * KD, KD, KD, (const float *)o->cd[l - 1], nin,
                                                  KD, (float *)o->cd[l], KD, SRC_PARENT, o->t_l2l, 8, nper, m2l_done ? 1 : 0,
                                                  o->l2l_scale[l], nullptr, want_of(o, l), false, st));
            } else {
                const T *A = ops.l2l + (size_t)(l - lmin - 1) * 8 * KD * KD;
                auto p = tap<T, T>(A, (int64_t)KD * KD, KD, KD, (T *)o->cd[l - 1], KD, (T *)o->cd[l], KD, SRC_PARENT,
                                   0, o->t_l2l, 8, npar, m2l_done ? 1 : 0);
                p.out_need = want_of(o, l);
                KIFMM_TRY(run(p, st));
            }
        }
        if (m2l_done) continue;
        PassTimer pt(o, KIFMM_PASS_M2L, st);
        KIFMM_TRY(m2l_level<T>(o, ops, l, precision, l > lmin ? 1 : 0, st));
    }
    if (fused_out) {   // the local expansions at the cells, plus the near field, in grid order
        KIFMM_HIP(hipStreamWaitEvent(st, o->join, 0));
        fj.side_forked = fj.fine_forked = false;
        PassTimer pt(o, KIFMM_PASS_L2P, st);
        if (precision == KIFMM_BF16X3)
            return run_l2p_permute_out_x3(*t, (const float *)o->cd[D], KD, o->l2p_xf, (const float *)SpN,
                                          (float)scale, want_of(o, D), (float *)S, st);
        return run_l2p_permute_out(*t, (const float *)o->cd[D], KD, o->l2p_frag, (const float *)SpN, (float)scale,
                                   want_of(o, D), (float *)S, st);
    }
    {
        PassTimer pt(o, KIFMM_PASS_L2P, st);
        // every leaf, also when targets are restricted: the wanted leaves then keep the
        // unrestricted values bit for bit (the others are written as zeros at the end; their
        // coefficients are finite, every level's coefficients being written in full)
        if (lowp) {
            const int64_t nin = nleaf * KD;
            if (precision == KIFMM_BF16)
                KIFMM_TRY(lowp_pass<__bf16>(o, o->l2pbf, 0, s, KD, (const float *)o->cd[D], nin, KD, (float *)Sp, s,
                                            SRC_SAME, o->t_single, 1, nleaf, 0, o->l2p_scale, nullptr, want_of(o, D),
                                            false, st));
            else
                KIFMM_TRY(lowp_pass<_Float16>(o, o->l2ph, 0, s, KD, (const float *)o->cd[D], nin, KD, (float *)Sp, s,
                                              SRC_SAME, o->t_single, 1, nleaf, 0, o->l2p_scale, nullptr, want_of(o, D),
                                              false, st));
        } else {
            auto p = tap<T, T>(ops.l2p, 0, s, KD, (T *)o->cd[D], KD, Sp, s, SRC_SAME, 0, o->t_single, 1, nleaf, 0);
            p.out_need = want_of(o, D);
            KIFMM_TRY(run(p, st));
        }
    }
    KIFMM_HIP(hipStreamWaitEvent(st, o->join, 0));
    fj.side_forked = fj.fine_forked = false;   // both joined into st (the fine stream before L2L into level D)
    PassTimer pt(o, KIFMM_PASS_PERMUTE_OUT, st);
    return launch_permute_out2<T>(*t, Sp, SpN, scale, want_of(o, D), S, st);
}

}  // namespace

extern "C" {

int kifmm_precompute_operators(kifmm_tree tree, const kifmm_kernel *kernel, const kifmm_opts *opts,
                               void *stream, kifmm_ops *out) {
    if (!tree || !out) return fail(KIFMM_EINVAL, "tree and out must be non-NULL");
    KIFMM_TRY(check_kernel(kernel));
    kifmm_opts o;
    if (opts) o = *opts;
    else { o.layout = KIFMM_LAYOUT_SINGLE; o.m0 = 6; o.check_edge = 10; o.rcond = 1e-7; o.lattice_radius = 0; }
    if (o.layout == KIFMM_LAYOUT_LATTICE && o.lattice_radius == 0) o.lattice_radius = 1.2;
    if (o.layout == KIFMM_LAYOUT_LATTICE && !(o.lattice_radius > 0.5 && o.lattice_radius <= 2.0))
        return fail(KIFMM_EINVAL, "lattice_radius must be in (0.5, 2]");
    if (o.layout < 0 || o.layout > 3) return fail(KIFMM_EINVAL, "unknown layout");
    if (o.layout == KIFMM_LAYOUT_LATTICE && (o.m0 < 3 || o.m0 > 8))
        return fail(KIFMM_EINVAL, "m0 must be in [3, 8] for the lattice layout");
    if (o.m0 < 2 || o.m0 > 16) return fail(KIFMM_EINVAL, "m0 must be in [2, 16]");
    if (o.layout != KIFMM_LAYOUT_PAPER && (o.check_edge < 2 || o.check_edge > 16))
        return fail(KIFMM_EINVAL, "check_edge must be in [2, 16]");
    if (!(o.rcond > 0 && o.rcond < 1)) return fail(KIFMM_EINVAL, "rcond must be in (0, 1)");
    kifmm_ops ops = new (std::nothrow) kifmm_ops_s();
    if (!ops) return fail(KIFMM_ENOMEM, "host allocation failed");
    ops->tree_magic = tree->magic;
    ops->D = tree->depth;
    ops->ell = tree->ell;
    ops->s = tree->s;
    ops->nb = tree->nb;
    ops->ellz = tree->ellz;
    ops->R = tree->R;
    // coarsest level with expansions: a cube's levels 0 and 1 have no interaction lists; on a
    // column of two cubes level 0 has none (the two roots are adjacent), from three on the
    // roots two or more apart interact at level 0
    ops->lmin = tree->R > 2 ? 0 : (tree->R == 2 ? 1 : 2);
    ops->kern = *kernel;
    ops->opts = o;
    int rc = build_ops(tree, ops, (hipStream_t)stream);
    if (rc != KIFMM_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        free_ops(ops);
        return rc;
    }
    *out = ops;
    return KIFMM_OK;
}

int kifmm_profile_enable(kifmm_ops ops, int32_t on) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    clear_profile(ops);
    if (!on) return KIFMM_OK;
    const int pairs = 4096;
    ops->ev.resize(2 * pairs);
    ops->ev_pass.assign(pairs, 0);
    for (auto &e : ops->ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            e = nullptr;
            ops->ev.resize(&e - ops->ev.data());
            clear_profile(ops);
            return hip_fail(r, "hipEventCreate");
        }
    }
    ops->prof = true;
    return KIFMM_OK;
}

int kifmm_profile_read(kifmm_ops ops, double *ms, int64_t *calls, int32_t n) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    drain_profile(ops);
    for (int p = 0; p < n && p < KIFMM_NPASS; ++p) {
        if (ms) ms[p] = ops->prof_ms[p];
        if (calls) calls[p] = ops->prof_calls[p];
    }
    return KIFMM_OK;
}

int kifmm_ops_skip_zero_sources(kifmm_ops ops, int32_t enable) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    if (!enable) {
        ops->skip_zero = false;
        return KIFMM_OK;
    }
    if (ops->D >= ops->lmin && ops->nz.empty()) {
        ops->nz.assign(ops->D + 1, nullptr);
        for (int l = ops->lmin; l <= ops->D; ++l) {
            const int rc = dmalloc(&ops->nz[l], (size_t)ops->R << (3 * l));
            if (rc != KIFMM_OK) {
                for (uint8_t *p : ops->nz)
                    if (p) (void)hipFree(p);
                ops->nz.clear();
                return rc;
            }
        }
    }
    ops->skip_zero = true;
    return KIFMM_OK;
}

int kifmm_ops_p2p_fft(kifmm_ops ops, int32_t enable) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    if (!enable) {
        ops->p2p_fft = false;
        return KIFMM_OK;
    }
    if (!ops->near_gh || ops->nb < 4)
        return fail(KIFMM_EUNSUPPORTED, "the Fourier-space near field needs leaves of 8^3 cells and at least 4 per axis");
    if (!ops->near_q) {
        const size_t n = (size_t)ops->nb * ops->nb * ops->nb * 1920 * 2;
        KIFMM_TRY(dmalloc(&ops->near_q, n));
        const int rc = dmalloc(&ops->near_p, n / 2);   // [nleaf][120][8]: after the x stage
        if (rc != KIFMM_OK) {
            (void)hipFree(ops->near_q);
            ops->near_q = nullptr;
            return rc;
        }
    }
    ops->p2p_fft = true;
    return KIFMM_OK;
}

int kifmm_ops_serial(kifmm_ops ops, int32_t enable) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    ops->serial = enable != 0;
    return KIFMM_OK;
}

int kifmm_ops_m2l_fft(kifmm_ops ops, int32_t enable) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    if (ops->opts.layout != KIFMM_LAYOUT_LATTICE) {
        if (!enable) return KIFMM_OK;
        return fail(KIFMM_EUNSUPPORTED, "the FFT form of M2L needs operators of the lattice layout");
    }
    ops->m2l_fft = enable != 0 && !ops->fft_g.empty();
    return KIFMM_OK;
}

int kifmm_ops_restrict_targets(kifmm_ops ops, const uint8_t *leaf_mask) {
    if (!ops) return fail(KIFMM_EINVAL, "ops is NULL");
    KIFMM_HIP(hipDeviceSynchronize());   // no evaluation may still read the old flags
    if (!leaf_mask) {
        for (uint8_t *p : ops->want)
            if (p) (void)hipFree(p);
        ops->want.clear();
        return KIFMM_OK;
    }
    const int D = ops->D, nb = ops->nb, R = ops->R;
    // host flags per level: leaves by root and Morton code, then each parent the OR of its 8
    // children
    std::vector<std::vector<uint8_t>> h(D + 1);
    const size_t nbz = (size_t)R * nb;
    h[D].assign((size_t)R * nb * nb * nb, 0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
            for (size_t c = 0; c < nbz; ++c)
                h[D][((c / nb) << (3 * D)) + morton_encode(a, b, (uint32_t)(c % nb))] =
                    leaf_mask[((size_t)a * nb + b) * nbz + c] != 0;
    for (int l = D - 1; l >= 0; --l) {
        h[l].assign((size_t)R << (3 * l), 0);
        for (size_t i = 0; i < h[l].size(); ++i)
            for (int k = 0; k < 8; ++k) h[l][i] |= h[l + 1][8 * i + k];
    }
    if (ops->want.empty()) {
        ops->want.assign(D + 1, nullptr);
        for (int l = 0; l <= D; ++l) {
            const int rc = dmalloc(&ops->want[l], h[l].size());
            if (rc != KIFMM_OK) {
                for (uint8_t *p : ops->want)
                    if (p) (void)hipFree(p);
                ops->want.clear();
                return rc;
            }
        }
    }
    for (int l = 0; l <= D; ++l)
        KIFMM_HIP(hipMemcpy(ops->want[l], h[l].data(), h[l].size(), hipMemcpyHostToDevice));
    return KIFMM_OK;
}

int kifmm_eval(kifmm_tree tree, kifmm_ops ops, const void *I_dev, double prefactor, void *S_dev,
               int32_t precision, void *stream) {
    if (!tree || !ops) return fail(KIFMM_EINVAL, "tree and ops must be non-NULL");
    if (ops->tree_magic != tree->magic) return fail(KIFMM_EMISMATCH, "ops were built for another tree");
    if (!I_dev || !S_dev) return fail(KIFMM_EINVAL, "I_dev and S_dev must be non-NULL");
    if (!std::isfinite(prefactor)) return fail(KIFMM_EINVAL, "prefactor must be finite");
    if (precision < KIFMM_FP64 || precision > KIFMM_FP16) return fail(KIFMM_EINVAL, "unknown precision");
    const size_t esz = precision == KIFMM_FP64 ? 8 : 4;
    const char *ib = (const char *)I_dev, *sb = (const char *)S_dev;
    const size_t bytes = (size_t)tree->N * esz;
    if (sb < ib + bytes && ib < sb + bytes) return fail(KIFMM_EINVAL, "I_dev and S_dev overlap");
    hipStream_t st = (hipStream_t)stream;
    if (ops->prof && 2 * (ops->ev_used + 64) > (int)ops->ev.size()) drain_profile(ops);
    if (precision == KIFMM_FP64)
        return eval_typed<double>(tree, ops, (const double *)I_dev, (double *)S_dev, prefactor, precision, st);
    return eval_typed<float>(tree, ops, (const float *)I_dev, (float *)S_dev, prefactor, precision, st);
}

}  // extern "C"
