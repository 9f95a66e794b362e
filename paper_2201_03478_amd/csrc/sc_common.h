// sc_common.h -- internal definitions shared by the HIP sources of libsidelobe.
//
// The plan holds the grid geometry and every device buffer of the two-step
// total-convolution method (Galloway et al. 2022, Sec. 2.1): ring sums of the
// Wigner-d recursion, the theta-upsampled ring spectra, the component maps on
// the oversampled grid, and the constant tables (transform twiddles, kernel
// deconvolution factors, recursion seed prefactors).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sidelobe.h"

#define SC_MAX_RADICES 16

// Radix schedule of one mixed-radix (2, 3, 4, 5) Stockham transform.  Stage s
// has radix r[s], span ns[s] = r[0] ... r[s-1] and twiddle stride
// tws[s] = n / (ns[s] r[s]); mag[s] = ceil(2^32 / ns[s]) turns j / ns[s] into a
// multiply-high (exact for j, ns < 2^16; unused when ns[s] = 1).
// Radix orders of the transform lengths that have compile-time kernels; the host
// plans use the same orders, so one pass-major twiddle table serves both.
#define SC_PLAN_540 9, 5, 12
#define SC_PLAN_1080 9, 12, 10
#define SC_PLAN_2160 15, 12, 12
#define SC_PLAN_4320 9, 5, 6, 16

struct FftPlan {
    int n;
    int nst;
    int r[SC_MAX_RADICES];
    int ns[SC_MAX_RADICES];
    int tws[SC_MAX_RADICES];
    unsigned mag[SC_MAX_RADICES];
};

// Default samples per work item of the binned gather, and samples per binning pass
// (a pass of 2^27 samples holds about 7.5 GB of binning workspace, 56 bytes per sample).
#define BIN_CHUNK 256
#define BIN_PASS_MAX (1 << 27)

// Anchor grid of the binned gather: key = row0 * nkc + col0.
struct BinGeom {
    double inv_hth, inv_hph;
    int n2os, nphi;
    int nkr, nkc;
};

// Samples in anchor order (structure of arrays).
// One binned sample, 32 bytes: u - floor(u) and v - floor(v) in grid units, psi
// reduced to [0, 2 pi), and the index of the sample within its pass.
struct __attribute__((aligned(32))) BinRec {
    double fu, fv, psi;
    int idx, pad;
};
// The same 32 bytes in FP32 adjoint passes, for the scatter: offsets in FP32 (what the
// scatter's weights use), e^{i psi} from FP64 sincos, and the sample's TOD gradient.
struct __attribute__((aligned(32))) AdjRec {
    float fu, fv;
    double cps, sps;
    float y;
    int idx;
};
static_assert(sizeof(AdjRec) == sizeof(BinRec), "adjoint records reuse the binning buffer");
struct BinSorted {
    BinRec *rec;  // in anchor order
};

// One detector's inputs to the persistent (batched) FP32 gather.
struct GatherDet {
    const int4 *items;
    const int *totals;
    BinSorted srt;
    const float *maps;
    float *tod;
    int cols, ncp, ncomp, nkc;
    float beta;
    int ct;  // component tiles (instantiated class)
};

#define SC_MAX_DET 64

struct BinWork {
    int64_t cap;      // samples per pass the buffers hold
    int64_t nkeys;
    int *count;       // [nkeys] samples per anchor
    int2 *offs;       // [nkeys] exclusive scan of (samples, items)
    int2 *sums;       // [scan blocks]
    int *totals;      // [4] samples, items, work cursor
    int *key, *rank;  // [cap]
    BinSorted sorted; // [cap]
    int4 *items;      // [cap] (key, first sorted sample, count, -)
    int64_t last_n;   // samples of the most recent binning pass
    size_t bytes;
};

struct sc_plan {
    int lmax, kmax, prec, W;
    double beta;       // exponential-of-semicircle shape parameter
    int nring;         // theta rings of the recursion, theta_j = (j + 1/2) pi / nring
    int n2;            // 2 nring: full-circle length of the forward theta transform
    int n2os;          // oversampled full-circle theta grid, spacing 2 pi / n2os
    int nphi;          // oversampled phi grid, spacing 2 pi / nphi
    int rows, cols;    // stored map rows (theta nodes incl. ghost rows) and columns (incl. wrap)
    int ncomp, ncp;    // 2 kmax + 2 stored components (cos/sin pairs), padded count
    int rpt, ngroups;  // recursion layout: rings per lane, ring groups per (k, m)
    int rpt_mx, ngroups_mx;  // the same for the FP32 (mixed-precision) recursion
    hipStream_t stream;
    hipStream_t side;             // sc_plan_convolve: binning beside the map synthesis
    hipEvent_t ev_fork, ev_join;  // (created on first use)
    hipEvent_t ev_stream;         // orders a new stream after the old one (sc_plan_set_stream)

    // Transform plans.  A transform longer than one workgroup's LDS (9216 points) runs as
    // sp* sub-transforms of length n / sp* (k_fft_big.hip); the plans and twiddle tables
    // below are those of the (sub-)transform length, n2, n2os and nphi the full lengths.
    FftPlan p2, p2os, pphi;
    int sp2, spos, spphi;
    int big;           // some transform is split: the k_fft_big.hip stages run
    double2 *S;        // big plans: theta spectra, [kmax+1][2 lmax+1][spad]
    int spad;          // padded row length of S (>= 2 lmax + 1)

    // Storage of the two spectral intermediates of the forward synthesis.  The FP32-map
    // forms (without split transforms) hold them as complex64: every value is still
    // computed in FP64 and rounded once on store, an error (2^-24 relative) of the
    // size the FP32 maps already carry, for half the bytes of the two largest
    // round trips through HBM.  The adjoint always uses them as complex128.
    int mid32;         // F and G hold float2 (forward path)
    int gst;           // row stride of G in elements: 2 lmax + 1, or 2 lmax + 2 with mid32

    // device buffers
    double2 *F;        // [kmax+1][2 lmax+1][nring] ring sums (float2 with mid32)
    double2 *G;        // [kmax+1][rows][gst] theta-upsampled, deconvolved (float2 with mid32)
    void *maps;        // column-tiled, float or double (sc_map_off)
    double2 *rroot;    // [lmax+1][lmax+1] at [x][l]: (sqrt((l+1)^2 - x^2), its reciprocal), 0 if l < x
    double4 *ctab;     // recursion coefficients (a, b, bn, S_l) of every (m, k, l), l >= max(m, k) (or null)
    long long *ctab_off;  // [lmax+1][kmax+1] first entry of each column
    double *sbin_m;    // [lmax+1][kmax+1] mantissa of sqrt(C(2 l, l + n))
    int *sbin_e;       // [lmax+1][kmax+1] binary exponent
    double *rtab;      // [nring][5] 1 - cos(theta_j); log2 cos(theta_j / 2), log2 sin(theta_j / 2) as (hi, lo) pairs
    double2 *tw2, *tw2os, *twphi;  // e^{-2 pi i t / N}
    double2 *phase;    // [2 lmax+1] e^{-i n pi / n2} / (n2 hhat_theta(n))
    double *dphi;      // [lmax+1] 1 / hhat_phi(m)
    double *glx, *glw; // Gauss-Legendre nodes/weights for the kernel transform
    int nq;

    int have_maps;
    size_t ws_bytes;
    BinWork bw;        // stream-ordered allocations (hipMallocAsync / hipFreeAsync on the plan's stream)
    void *gmaps;       // adjoint: gradient maps, [rows][cols][ncp] in both precisions (allocated on first use)
    double2 *GA;       // adjoint: per-k gradient contributions [kmax+1][n_alm]
    double2 *GB;       // beam adjoint: per-m gradient contributions [lmax+1][n_blm] (allocated on first use)
    size_t adj_bytes;
    int alm_lmax;          // band limit of the sky array's layout (>= lmax; a shared sky may be larger)
    int bin_fixed;         // binning buffers are referenced by a batch: never reallocate them
    int bin_chunk;         // samples per gather work item (tunable)
    int gather_wgs_per_cu; // persistent gather workgroups per CU (0: as many as fit; tunable)
    int gather_waves;      // waves per matrix-core gather workgroup, 4 or 8 (tunable)
    int gather_mma;        // matrix-core product form, SC_MMA_FP32 or SC_MMA_SPLIT16
    int gather_direct;     // force the per-sample gather (env SC_GATHER_PATH=direct)
    int gather_valu;       // FP32 binned gather on the VALU instead of MFMA (env SC_GATHER_PATH=valu)
    int64_t bin_pass_max;  // samples per binning pass (env SC_BIN_PASS_MAX, default BIN_PASS_MAX)

    // per-kernel event timing (see sc_plan_enable_timing)
    // psi cube (the paper's second step): [rows][cols][npst], built on request
    int npsi, npst;        // psi grid points; stored per pixel (npsi + W - 1 with halo, padded to 4)
    FftPlan ppsi;
    double2 *twpsi;        // pass-major twiddles of the npsi-point transform
    double *gpsi;          // [kmax+1] 1 / hhat_psi(k)
    void *cube;        // twpsi, gpsi and cube: stream-ordered allocations like bw
    int have_cube;
    int timing;
    int validate;  // SC_PARAM_VALIDATE: count non-finite inputs before launching (synchronous)
    int det_adjoint;   // SC_PARAM_DETERMINISTIC: atomic-free scatter (patch gradients, fixed-order sums)
    float *pg;         // its patch gradients [items][64 taps][16 CT]
    size_t pg_bytes;
    int *vcount;   // its device counter (allocated on first use)
    struct TimedLaunch *tl;  // pool of event pairs
    int tl_n, tl_cap;
};

enum { SC_STAGE_RING = 0, SC_STAGE_THETA = 1, SC_STAGE_PHI = 2, SC_STAGE_GATHER = 3, SC_STAGE_BIN = 4,
       SC_STAGE_SCATTER = 5, SC_STAGE_ADJ_FFT = 6, SC_STAGE_ADJ_RING = 7, SC_NSTAGE = 8 };

struct TimedLaunch {
    int stage;
    hipEvent_t a, b;
};

static inline size_t sc_map_elem_bytes(const sc_plan *p) { return p->prec == SC_FP64 ? 8 : 4; }

// Storage order of the component maps: column-tiled in groups of 16 bytes of
// components (G = 4 floats or 2 doubles).  Value (row r, column c, component q)
// sits at ((r ntile + c / 8) (ncp / G) + q / G) 8 G + (c mod 8) G + q mod G,
// ntile = ceil(cols / 8): a group's values at eight consecutive columns are 128
// contiguous bytes (for FP32 maps the four values of one k pair, components 4g ..
// 4g + 3; for FP64 maps the cos/sin pair of one k), so the phi synthesis of a k
// group writes whole lines, and the gather reads a group's 8 x 8 block as eight
// 128-byte runs.  ncp is a multiple of 16 for FP32 maps and of 4 for FP64 maps.
__host__ __device__ __forceinline__ int sc_map_ntile(int cols) { return (cols + 7) >> 3; }
// FP32 maps, in floats: q4 = q / 4, ng = ncp / 4
__device__ __forceinline__ size_t sc_tile_off(int r, int c, int q4, int ntile, int ng) {
    return ((((size_t)r * ntile + (c >> 3)) * ng + q4) << 5) + ((c & 7) << 2);
}
template <typename T>
__device__ __forceinline__ size_t sc_map_off(int r, int c, int q, int cols, int ncp) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "float or double maps");
    constexpr int LG = sizeof(T) == 4 ? 2 : 1;  // log2 of the group size G
    return ((((size_t)r * sc_map_ntile(cols) + (c >> 3)) * (size_t)(ncp >> LG) + (q >> LG)) << (LG + 3)) +
           ((c & 7) << LG) + (q & ((1 << LG) - 1));
}
// bytes of the plan's map buffer (FP32: whole tiles of eight columns)
static inline size_t sc_map_bytes(const sc_plan *p) {
    return sc_map_elem_bytes(p) * (size_t)p->rows * (8 * (size_t)sc_map_ntile(p->cols)) * p->ncp;
}

// ---------------------------------------------------------------- launchers
hipError_t sc_launch_tables(sc_plan *p);
// the maps in (row, column, component) order into dst (rows x cols x ncp values)
hipError_t sc_launch_maps_rowmajor(sc_plan *p, void *dst);
hipError_t sc_launch_psi_tables(sc_plan *p);
hipError_t sc_launch_psi_cube(sc_plan *p);
hipError_t sc_launch_gather_psi(sc_plan *p, const double *ptg, int64_t n, void *tod);
int sc_psi_max_len();
hipError_t sc_launch_ring_sums(sc_plan *p, const double *alm, const double *blm);
hipError_t sc_launch_rec_table(sc_plan *p);  // fills ctab (after sc_launch_tables)
void sc_choose_ring_layout(int nring, int *rpt, int *ngroups);
int sc_ring_groups(int nring, int rpt);  // ring groups of the FP64 ring-sum kernel
hipError_t sc_launch_ring_sums_mixed(sc_plan *p, const double *alm, const double *blm);
void sc_choose_ring_layout_mixed(int nring, int *rpt, int *ngroups);
hipError_t sc_launch_theta_upsample(sc_plan *p);
hipError_t sc_launch_theta_upsample_big(sc_plan *p);
hipError_t sc_launch_widen(const float2 *src, double2 *dst, size_t n, hipStream_t s);  // complex64 -> complex128
hipError_t sc_launch_phi_synthesis_big(sc_plan *p);
hipError_t sc_launch_phi_adjoint_big(sc_plan *p, const void *gmaps);
hipError_t sc_launch_theta_adjoint_big(sc_plan *p);
hipError_t sc_launch_phi_synthesis(sc_plan *p);
hipError_t sc_launch_phi_adjoint(sc_plan *p, const void *gmaps);
hipError_t sc_launch_theta_adjoint(sc_plan *p);
hipError_t sc_launch_ring_sums_adjoint(sc_plan *p, const double *blm, double *grad);
int sc_adjoint_slabs(const sc_plan *p);  // ring slabs per column of the adjoint recursion
hipError_t sc_launch_ring_sums_adjoint_beam(sc_plan *p, const double *alm, double *grad);
hipError_t sc_launch_scatter(sc_plan *p, const double *ptg, int64_t n, const void *y, void *gmaps);
hipError_t sc_launch_scatter_binned(sc_plan *p, void *gmaps);  // after sc_launch_binning with y
hipError_t sc_launch_scatter_reduce(sc_plan *p, void *gmaps);  // deterministic mode, after the scatter
hipError_t sc_launch_det_order(sc_plan *p, int nitems);         // deterministic mode, after the binning
int sc_det_max_items();                                         // largest anchor it orders
bool sc_scatter_binned_supported(const sc_plan *p);
hipError_t sc_launch_zero(void *dst, size_t bytes, hipStream_t stream);
// Adds to *count the number of NaN or infinite values among x[0 .. n) (double, or float with f32).
hipError_t sc_launch_count_nonfinite(const void *x, int64_t n, int f32, int *count, hipStream_t stream);
hipError_t sc_launch_gather(sc_plan *p, const double *ptg, int64_t n, void *tod);
// Sort samples into anchor order (k_bin.hip).  With y (FP32 adjoint passes) the
// records take the adjoint layout AdjRec instead of BinRec.
hipError_t sc_launch_binning(sc_plan *p, const double *ptg, int64_t n, const float *y = nullptr);
hipError_t sc_launch_dipole(const double *blm, int lmax, int kmax, const double *ptg, int64_t n, const double *beta,
                            int64_t spp, double T0, double q, double *out, hipStream_t stream);
hipError_t sc_launch_gather_binned(sc_plan *p, void *tod);
bool sc_gather_mfma64_supported(int W);
hipError_t sc_launch_gather_mfma64(sc_plan *p, void *tod);
GatherDet sc_gather_det(const sc_plan *p, void *tod);
hipError_t sc_launch_gather_batch(const GatherDet *dets_dev, int ndet, int max_ct, int *cursor, int wgs_per_cu, int waves,
                                  int mma, hipStream_t stream);
bool sc_gather_binned_supported(const sc_plan *p);

static inline BinGeom sc_bin_geom(const sc_plan *p) {
    const double two_pi = 6.283185307179586477;
    BinGeom g;
    g.inv_hth = (double)p->n2os / two_pi;
    g.inv_hph = (double)p->nphi / two_pi;
    g.n2os = p->n2os;
    g.nphi = p->nphi;
    g.nkr = p->n2os / 2 + 1;
    g.nkc = p->nphi;
    return g;
}

// Host-side helpers of sc_api.cpp: the calling thread's error message (sc_last_error),
// and the argument checks and path choice of an interpolation.
int sc_error(int code, const char *fmt, ...);
int sc_hip_error(hipError_t e, const char *what);
void sc_clear_error();
int sc_check_interp_args(sc_plan *p, const double *ptg, void *tod);
bool sc_uses_binning(const sc_plan *p);

// Set a kernel's dynamic-LDS limit once (cached; safe to call while a stream is
// being captured into a graph, since a cached call makes no runtime call).
hipError_t sc_set_lds_attr(const void *kern, size_t lds);
// Workgroups of a persistent launch: occupancy per CU (optionally capped) x CUs (cached).
int sc_persistent_grid(const void *kern, int block, size_t lds, int wgs_per_cu);

// ------------------------------------------------------------ device helpers
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap the hardware block index so that consecutive logical indices run on
// the same XCD at about the same time: their partial-line writes to
// neighbouring addresses then merge in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int x = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Blocks (column, ring group) of a launch with ng groups per column: the ng
// blocks of one column run on one XCD at about the same time, so the column's
// coefficients and weights are fetched from HBM once and the other groups find
// them in that XCD's L2; consecutive columns go round-robin over the XCDs.
__device__ __forceinline__ void xcd_column_group(int b, int ncol, int ng, int &col, int &g) {
    const int span = 8 * ng;
    const int full = (ncol >> 3) * span;  // blocks of whole 8-column chunks
    if (b < full) {
        const int c8 = b / span, r = b - c8 * span;
        g = r >> 3;
        col = 8 * c8 + (r & 7);  // XCD b % 8 = col % 8 for every group
    } else {
        const int r = b - full;
        col = (ncol & ~7) + r / ng;
        g = r - (r / ng) * ng;
    }
}

// Exponential-of-semicircle tap weight in FP32, exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1
// and 0 outside, evaluated as 2^(-beta log2(e) z^2 / (1 + sqrt(1 - z^2))): the same function
// without the cancellation of sqrt(1 - z^2) - 1 next to z = 0, where the weights are largest.
// nbl = -beta log2(e).  Hardware square root, reciprocal and exp2 (about 1 ulp each): the
// exponent carries a relative error of a few ulp, so the weight's relative error is below
// 1e-7 plus 2.4e-7 times its |log2|, i.e. an absolute error under 1e-7 at every z.
__device__ __forceinline__ float es_weight_f32(float z, float nbl) {
    const float z2 = z * z;
    const float q = __builtin_fmaf(-z, z, 1.f);
    if (!(q > 0.f)) return 0.f;
    const float s = __builtin_amdgcn_sqrtf(q);
    return __builtin_amdgcn_exp2f(nbl * z2 * __builtin_amdgcn_rcpf(1.f + s));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Loads and stores of complex values held as complex128 or complex64 (computed in FP64).
__device__ __forceinline__ double2 ld2(const double2 *p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2 *p) {
    const float2 v = *p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2 *p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
