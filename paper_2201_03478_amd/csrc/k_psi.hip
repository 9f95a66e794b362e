// k_psi.hip -- the paper's second step: the cube c(theta, phi, psi) on a psi
// grid, and three-dimensional interpolation of it at the pointings.
//
// The two-step algorithm of Galloway et al. 2022 (Sec. 2.1) first builds, for
// every k, the spin-k map, and then takes, on every (theta, phi) grid point, the
// Fourier series over k onto a grid in psi, so that the signal at any pointing
// is an interpolation of one real cube.  Here the psi grid has npsi points,
// psi_j = 2 pi j / npsi with npsi >= 2 (2 kmax + 1) (the same twofold
// oversampling as the phi grid), and the series is divided by the transform
// of the interpolation kernel so that interpolating the cube with it
// reproduces the series (the deconvolution of Sec. 2.1 applied along psi):
//     cube(r, q, j) = sum_{k <= kmax} g_k (M_2k(r, q) cos k psi_j + M_2k+1(r, q) sin k psi_j),
//     g_k = 1 / hhat_psi(k),
// with M_c the stored component maps (cos / sin pair of k at 2k, 2k + 1).
//
// Cube layout: [row][col][npst], psi fastest.  Entry s of a pixel holds grid
// point (s - W/2 + 1) mod npsi for s < npsi + W - 1 (a periodic halo, so the W
// psi nodes of a sample are W consecutive values), zero beyond.
//
// Build: one transform per two pixels (a wave, or 16 or 32 lanes of one for short psi
// grids).  The series of a pixel is real, so its
// spectrum is Hermitian: Y(k) = g_k (M_2k - i M_2k+1) / 2 at +k, the conjugate at
// -k, g_0 M_0 at 0.  Two pixels a, b share one complex inverse transform of
// X = Y_a + i Y_b, whose output is c_a + i c_b.  The transform is the LDS
// Stockham FFT (fft_lds.h) in FP64; values are stored in the map type.
#include "fft_lds.h"

namespace {

constexpr int PSI_NT = 64;  // lanes per wave, shared by G transforms
constexpr int PSI_PT = 8;   // npsi <= 512

constexpr int PSI_SLACK = 512;  // zeroed bytes after the cube (reached by the last pixel's quad reads)

// Map values of one pixel pair at a lane's two orders k = tg, tg + NTS (tg: the lane's index
// among the NTS lanes of its transform): (M_2k, M_2k+1) of pixel a, then of pixel b (zero past
// kmax and for a missing b).  Two orders per lane suffice: kmax + 1 <= npsi / 4 <= 2 NTS.
template <typename T, int NTS>
__device__ __forceinline__ void fetch_pair(const T *__restrict__ maps, int64_t pair, int64_t npix, int cols, int ncp,
                                           int kmax, int tg, T (&r)[8]) {
    const int64_t a = 2 * pair;
    const bool hb = a + 1 < npix;
    // pixels are (row, column) in row-major order; rows x cols < 2^31 up to lmax 8192
    const unsigned ua = (unsigned)a, ub = hb ? ua + 1u : ua, uc = (unsigned)cols;
    const int ra = (int)(ua / uc), ca = (int)(ua - (unsigned)ra * uc);
    const int rb = (int)(ub / uc), cb = (int)(ub - (unsigned)rb * uc);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = tg + NTS * h;
        const bool ok = k <= kmax;
        const size_t oa = sc_map_off<T>(ra, ca, ok ? 2 * k : 0, cols, ncp);
        const size_t ob = sc_map_off<T>(rb, cb, ok ? 2 * k : 0, cols, ncp);
        r[4 * h] = ok ? maps[oa] : (T)0;
        r[4 * h + 1] = ok ? maps[oa + 1] : (T)0;
        r[4 * h + 2] = ok && hb ? maps[ob] : (T)0;
        r[4 * h + 3] = ok && hb ? maps[ob + 1] : (T)0;
    }
}

// Persistent over pixel pairs, two waves per workgroup sharing the twiddle table; each wave
// runs G transforms side by side (NTS = 64 / G lanes each, G = 1 for lengths above 128), so
// short psi grids still fill the wave.  Iteration it of a workgroup covers pairs
// (2 it + w) G + g for wave w and transform g.  The next pairs' map values are loaded before
// the current transforms so that the load latency overlaps them.  Twiddles and the
// deconvolution factors are read once per workgroup (LDS, registers): no global loads inside
// the transform.  Every transform runs in every iteration (its barriers are the workgroup's);
// one without a pair in the last iteration transforms stale values and stores nothing.
template <typename T, typename S, int G>
__global__ void __launch_bounds__(2 * PSI_NT)
k_psi_cube(const T *__restrict__ maps, T *__restrict__ cube, int64_t npix, int cols, int ncp, int kmax, int npsi, int npst,
           int W, FftPlan P, const double2 *__restrict__ tw, const double *__restrict__ gpsi) {
    constexpr int NTS = PSI_NT / G;   // lanes per transform
    constexpr int PTS = PSI_PT * G;   // points per lane: NTS PTS = 512
    constexpr int NB = FftLen<S>::value > 0 ? FftLen<S>::value : PSI_NT * PSI_PT / G;  // LDS per transform
    static_assert(G == 1 || FftLen<S>::value > 0, "several transforms per wave need a compile-time plan");
    __shared__ double2 bufs[2][G][NB];
    __shared__ double2 twl[NB];
    const int lane = threadIdx.x & (PSI_NT - 1), wv = threadIdx.x / PSI_NT;
    const int g = lane / NTS, tg = lane - g * NTS;
    double2 *buf = bufs[wv][g];
    const int half = W / 2;
    const int ext = npsi + W - 1;
    const int64_t npairs = (npix + 1) / 2;
    for (int t = threadIdx.x; t < npsi; t += 2 * PSI_NT) twl[t] = tw[t];
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < PSI_SLACK / (int)sizeof(T); e += 2 * PSI_NT) cube[npix * npst + e] = (T)0;
    double gk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = tg + NTS * h;
        gk[h] = k > kmax ? 0.0 : (k == 0 ? gpsi[0] : 0.5 * gpsi[k]);
    }
    // consecutive pairs share the 128-byte lines of the column-tiled maps: the workgroups
    // that take them start on one XCD (xcd_remap is a permutation of the block indices)
    int64_t it = xcd_remap(blockIdx.x, gridDim.x);
    T nxt[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) nxt[e] = (T)0;
    if ((2 * it + wv) * G + g < npairs) fetch_pair<T, NTS>(maps, (2 * it + wv) * G + g, npix, cols, ncp, kmax, tg, nxt);
    for (; 2 * it * G < npairs; it += gridDim.x) {
        const int64_t pair = (2 * it + wv) * G + g;
        T cur[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) cur[e] = nxt[e];
        const int64_t pn = (2 * (it + gridDim.x) + wv) * G + g;
        if (pn < npairs) fetch_pair<T, NTS>(maps, pn, npix, cols, ncp, kmax, tg, nxt);
        for (int t = tg; t < npsi; t += NTS)
            if (t > kmax && t < npsi - kmax) buf[t] = make_double2(0.0, 0.0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = tg + NTS * h;
            if (k <= kmax) {
                const double gg = gk[h];
                const double ca = (double)cur[4 * h], sa = (double)cur[4 * h + 1];
                const double cb = (double)cur[4 * h + 2], sb = (double)cur[4 * h + 3];
                // +k: Y_a + i Y_b with Y = g (M_2k - i M_2k+1); -k: the conjugates
                buf[k] = make_double2(gg * (ca + sb), gg * (cb - sa));
                if (k > 0) buf[npsi - k] = make_double2(gg * (ca - sb), gg * (cb + sa));
            }
        }
        __syncthreads();
        FftRun<+1, NTS, PTS, S>::run(buf, P, twl, tg, NTS);
        if (pair < npairs) {
            const int64_t a = 2 * pair, b = a + 1;
            const bool hb = b < npix;
            for (int s2 = tg; s2 < npst; s2 += NTS) {
                int j = s2 - half + 1;
                j = j < 0 ? j + npsi : (j >= npsi ? j - npsi : j);
                const double2 v = s2 < ext ? buf[j] : make_double2(0.0, 0.0);
                cube[a * npst + s2] = (T)v.x;
                if (hb) cube[b * npst + s2] = (T)v.y;
            }
        }
        __syncthreads();
    }
}

// exp(beta (sqrt(1 - z^2) - 1)) without the cancellation next to z = 0
template <typename T>
__device__ __forceinline__ T es_w(T z, T beta) {
    const T z2 = z * z, q = (T)1 - z2;
    return q > (T)0 ? exp(-beta * z2 / ((T)1 + sqrt(q))) : (T)0;
}

// Grid coordinate in [0, n) of an angle on a periodic grid of n points.
__device__ __forceinline__ double periodic_coord(double a, double inv_h, int n) {
    const double two_pi = 6.283185307179586477;
    double v = (a - two_pi * floor(a / two_pi)) * inv_h;
    if (!(v < (double)n)) v = 0.0;  // 2 pi rounding, NaN
    return v < 0.0 ? 0.0 : v;
}

// One thread per sample: W^3 products of separable kernel weights with the cube.
// Grid indices and fractional offsets in FP64, as in the two-dimensional gather.
template <typename T, int W>
__global__ void __launch_bounds__(256)
k_gather_psi(const double *__restrict__ ptg, int64_t n, const T *__restrict__ cube, T *__restrict__ tod, int cols,
             int npst, double beta, double inv_hth, double inv_hph, double inv_hps, int n2os, int nphi, int npsi) {
    constexpr int half = W / 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
        double u = th * inv_hth;
        u = fmin(fmax(u, 0.0), 0.5 * (double)n2os);
        const int r0 = (int)floor(u) - half + 1;
        const double v = periodic_coord(ph, inv_hph, nphi);
        const int q0 = (int)floor(v) - half + 1;
        const double x = periodic_coord(ps, inv_hps, npsi);
        const int p0 = (int)floor(x) - half + 1;
        T wt[W], wp[W], wq[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            wt[i] = es_w<T>((T)((u - (double)(r0 + i)) / half), (T)beta);
            wp[i] = es_w<T>((T)((v - (double)(q0 + i)) / half), (T)beta);
            wq[i] = es_w<T>((T)((x - (double)(p0 + i)) / half), (T)beta);
        }
        const T *base = cube + ((size_t)(r0 + half - 1) * cols + (size_t)(q0 + half - 1)) * npst + (p0 + half - 1);
        T acc = (T)0;
        for (int i = 0; i < W; ++i) {
            T ai = (T)0;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const T *c = base + ((size_t)i * cols + j) * npst;
                T t = (T)0;
#pragma unroll
                for (int l = 0; l < W; ++l) t += wq[l] * c[l];
                ai += wp[j] * t;
            }
            acc += wt[i] * ai;
        }
        tod[s] = acc;
    }
}

// FP32 cube: each run of W psi values is read as (W + 6) / 4 aligned float4 quads from the
// quad boundary at or below its first entry.  The weights are evaluated at the nodes of all
// 4 NQ entries: the kernel vanishes at |z| >= 1, so the entries outside the W-point stencil
// get weight 0 and the stencil's own weights are the same values as above.  The last quad
// can reach past the pixel's npst entries into the next pixel (finite values, weight 0) or,
// for the last pixel, into the zeroed slack after the cube.
// With a sample order (the binning's records in anchor order), thread t takes sample
// order[t].idx instead of t: samples that share a stencil anchor run together and reuse
// the same cube lines from cache.  Each sample's arithmetic is unchanged.
template <int W>
__global__ void __launch_bounds__(256)
k_gather_psi_f32(const double *__restrict__ ptg, int64_t n, const float *__restrict__ cube, float *__restrict__ tod,
                 int cols, int npst, double beta, double inv_hth, double inv_hph, double inv_hps, int n2os, int nphi,
                 int npsi, const BinRec *__restrict__ order) {
    constexpr int half = W / 2;
    constexpr int NQ = (W + 6) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int64_t s = order ? (int64_t)order[t].idx : t;
        const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
        double u = th * inv_hth;
        u = fmin(fmax(u, 0.0), 0.5 * (double)n2os);
        const int r0 = (int)floor(u) - half + 1;
        const double v = periodic_coord(ph, inv_hph, nphi);
        const int q0 = (int)floor(v) - half + 1;
        const double x = periodic_coord(ps, inv_hps, npsi);
        const int a0 = ((int)floor(x)) & ~3;  // stored index of the first psi entry, rounded down to a quad
        float wt[W], wp[W], wq[4 * NQ];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            wt[i] = es_w<float>((float)((u - (double)(r0 + i)) / half), (float)beta);
            wp[i] = es_w<float>((float)((v - (double)(q0 + i)) / half), (float)beta);
        }
#pragma unroll
        for (int m = 0; m < 4 * NQ; ++m)  // stored entry a0 + m holds grid node a0 + m - half + 1
            wq[m] = es_w<float>((float)((x - (double)(a0 + m - half + 1)) / half), (float)beta);
        const float4 *base =
            (const float4 *)(cube + ((size_t)(r0 + half - 1) * cols + (size_t)(q0 + half - 1)) * npst + a0);
        const size_t rq = (size_t)npst / 4;
        float acc = 0.0f;
        for (int i = 0; i < W; ++i) {
            float ai = 0.0f;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const float4 *c = base + ((size_t)i * cols + j) * rq;
                float t = 0.0f;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const float4 c4 = c[q];
                    t += wq[4 * q] * c4.x + wq[4 * q + 1] * c4.y + wq[4 * q + 2] * c4.z + wq[4 * q + 3] * c4.w;
                }
                ai += wp[j] * t;
            }
            acc += wt[i] * ai;
        }
        tod[s] = acc;
    }
}

template <typename T, int W>
void launch_gather_psi(const sc_plan *p, const double *ptg, int64_t n, void *tod, unsigned nblk,
                       const BinRec *order) {
    const double two_pi = 6.283185307179586477;
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((k_gather_psi_f32<W>), dim3(nblk), dim3(256), 0, p->stream, ptg, n,
                           (const float *)p->cube, (float *)tod, p->cols, p->npst, p->beta, (double)p->n2os / two_pi,
                           (double)p->nphi / two_pi, (double)p->npsi / two_pi, p->n2os, p->nphi, p->npsi, order);
    else
        hipLaunchKernelGGL((k_gather_psi<T, W>), dim3(nblk), dim3(256), 0, p->stream, ptg, n, (const T *)p->cube,
                           (T *)tod, p->cols, p->npst, p->beta, (double)p->n2os / two_pi, (double)p->nphi / two_pi,
                           (double)p->npsi / two_pi, p->n2os, p->nphi, p->npsi);
}

template <typename T>
void launch_gather_psi_w(const sc_plan *p, const double *ptg, int64_t n, void *tod, unsigned nblk,
                         const BinRec *order) {
    switch (p->W) {
        case 4: launch_gather_psi<T, 4>(p, ptg, n, tod, nblk, order); break;
        case 6: launch_gather_psi<T, 6>(p, ptg, n, tod, nblk, order); break;
        case 8: launch_gather_psi<T, 8>(p, ptg, n, tod, nblk, order); break;
        case 10: launch_gather_psi<T, 10>(p, ptg, n, tod, nblk, order); break;
        case 12: launch_gather_psi<T, 12>(p, ptg, n, tod, nblk, order); break;
        case 14: launch_gather_psi<T, 14>(p, ptg, n, tod, nblk, order); break;
        default: launch_gather_psi<T, 16>(p, ptg, n, tod, nblk, order); break;
    }
}

// psi transforms with their passes fixed at compile time, for kmax = 100, 32 and 16 (npsi = 405,
// 135, 72); the shorter ones run 2 and 4 transforms per wave.  Other lengths take the
// runtime-planned transform, one per wave.  The radix orders are the ones factor_fft plans,
// so both forms read the same twiddle table.
using PsiSpec405 = FftSpec<405, 9, 9, 5>;
using PsiSpec135 = FftSpec<135, 9, 15>;
using PsiSpec72 = FftSpec<72, 9, 8>;

bool plan_is(const FftPlan &P, int n, int r0, int r1, int r2) {
    return P.n == n && P.nst == (r2 ? 3 : 2) && P.r[0] == r0 && P.r[1] == r1 && (!r2 || P.r[2] == r2);
}

template <typename T, typename S, int G>
void launch_psi_cube(sc_plan *p, int64_t npix) {
    const int64_t iters = ((npix + 1) / 2 + 2 * G - 1) / (2 * G);  // 2 G pixel pairs per workgroup iteration
    const unsigned nblk = (unsigned)(iters < 16384 ? iters : 16384);
    hipLaunchKernelGGL((k_psi_cube<T, S, G>), dim3(nblk), dim3(2 * PSI_NT), 0, p->stream, (const T *)p->maps,
                       (T *)p->cube, npix, p->cols, p->ncp, p->kmax, p->npsi, p->npst, p->W, p->ppsi, p->twpsi, p->gpsi);
}

template <typename T>
void launch_psi_cube_any(sc_plan *p, int64_t npix) {
    if (plan_is(p->ppsi, 405, 9, 9, 5))
        launch_psi_cube<T, PsiSpec405, 1>(p, npix);
    else if (plan_is(p->ppsi, 135, 9, 15, 0))
        launch_psi_cube<T, PsiSpec135, 2>(p, npix);
    else if (plan_is(p->ppsi, 72, 9, 8, 0))
        launch_psi_cube<T, PsiSpec72, 4>(p, npix);
    else
        launch_psi_cube<T, FftGeneric, 1>(p, npix);
}

}  // namespace

int sc_psi_max_len() { return PSI_NT * PSI_PT; }
int sc_psi_slack_bytes() { return PSI_SLACK; }

hipError_t sc_launch_psi_cube(sc_plan *p) {
    const int64_t npix = (int64_t)p->rows * p->cols;
    if (p->prec == SC_FP64)
        launch_psi_cube_any<double>(p, npix);
    else
        launch_psi_cube_any<float>(p, npix);
    return hipGetLastError();
}

static hipError_t gather_psi(sc_plan *p, const double *ptg, int64_t n, void *tod, const BinRec *order) {
    if (n == 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (p->prec == SC_FP64)
        launch_gather_psi_w<double>(p, ptg, n, tod, (unsigned)nb, nullptr);
    else
        launch_gather_psi_w<float>(p, ptg, n, tod, (unsigned)nb, order);
    return hipGetLastError();
}

hipError_t sc_launch_gather_psi(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    return gather_psi(p, ptg, n, tod, nullptr);
}

// FP32 cube, samples in the order of the plan's most recent binning pass over these n pointings.
hipError_t sc_launch_gather_psi_sorted(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    return gather_psi(p, ptg, n, tod, p->bw.sorted.rec);
}
