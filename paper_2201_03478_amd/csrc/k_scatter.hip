// k_scatter.hip -- adjoint of the interpolation + k-sum (scatter to gradient maps).
//
// The gather computes c_t = sum_{taps} w_t(tap) sum_c basis_c(psi_t) M_c[tap]
// (k_gather.hip).  Its adjoint for a TOD gradient y is
//     GM_c[p] = sum_t y_t w_t(p) basis_c(psi_t)
// over the samples whose stencil covers map pixel p.  Different samples and
// anchors add into the same pixels, so the result is accumulated with
// hardware floating-point atomics (order-dependent rounding, Z15).
//
//  * k_scatter_mfma (FP32 maps, W = 8): per work item (samples of one anchor,
//    k_bin.hip) the 64 x ncomp patch gradient PG[t][c] = sum_s w_s(t) V[s][c],
//    V[s][c] = y_s basis_c(psi_s), is a v_mfma_f32_16x16x4_f32 product summed
//    over all chunks of the item, then added to the maps with one atomic per
//    (tap, component).  Each sample's record (the binning's adjoint layout, with
//    e^{i psi} and the TOD gradient) is read once, by one thread, and the tap
//    weight w_s(t) = w_theta(t / 8) w_phi(t % 8) is formed from the 1-d weights
//    in LDS as the matrix operand is read.  The atomics are not what limits it:
//    without them the kernel takes within 2% of the time.
//  * k_scatter_direct (any W, FP32 or FP64): one wave per sample, lanes over
//    components, one atomic per (tap, component, sample).
#include "sc_common.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

// exp(beta (sqrt(1 - z^2) - 1)) without the cancellation next to z = 0
template <typename T>
__device__ __forceinline__ T es_w(T z, T beta) {
    const T z2 = z * z, q = (T)1 - z2;
    return q > (T)0 ? exp(-beta * z2 / ((T)1 + sqrt(q))) : (T)0;
}

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ double2 cpow_int(double2 z, int n) {
    double2 r = make_double2(1.0, 0.0);
    while (n) {
        if (n & 1) r = cmul(r, z);
        z = cmul(z, z);
        n >>= 1;
    }
    return r;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_scatter_direct(const double *__restrict__ ptg, int64_t n, const T *__restrict__ y, T *__restrict__ gmaps, int cols,
                 int ncp, int ncomp, int W, double beta, double inv_hth, double inv_hph, int n2os, int nphi) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int half = W / 2;
    const double two_pi = 6.283185307179586477;
    for (int64_t s = wave; s < n; s += nwaves) {
        const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
        double u = th * inv_hth;
        u = fmin(fmax(u, 0.0), 0.5 * (double)n2os);
        const int r0 = (int)floor(u) - half + 1;
        double v = (ph - two_pi * floor(ph / two_pi)) * inv_hph;
        if (!(v < (double)nphi) || v < 0.0) v = 0.0;
        const int q0 = (int)floor(v) - half + 1;
        T w = (T)0;
        if (lane < W)
            w = es_w<T>((T)((u - (double)(r0 + lane)) / half), (T)beta);
        else if (lane < 2 * W)
            w = es_w<T>((T)((v - (double)(q0 + lane - W)) / half), (T)beta);
        const double psr = ps - two_pi * floor(ps / two_pi);
        const T ys = y[s];
        T val[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = lane + 64 * t;
            T bas = (T)0;
            if (c < ncomp) {
                double sn, cs;
                sincos((double)(c >> 1) * psr, &sn, &cs);
                bas = (T)((c & 1) ? sn : cs);
            }
            val[t] = ys * bas;
        }
        const int row0 = r0 + half - 1, col0 = q0 + half - 1;
        for (int i = 0; i < W; ++i) {
            const T wi = __shfl(w, i);
            for (int j = 0; j < W; ++j) {
                const T wij = wi * __shfl(w, W + j);
                T *base = gmaps + ((size_t)(row0 + i) * cols + (col0 + j)) * ncp;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = lane + 64 * t;
                    if (c < ncomp && c != 1) atomic_add(base + c, wij * val[t]);  // basis_1 = sin 0 = 0
                }
            }
        }
    }
}

constexpr int W1ROW = 65;  // row stride of the 1-d weights: the 8 phi rows of one sample in distinct banks

template <int CT>
struct ScatterLds {
    static constexpr int NC = 16 * CT;
    static constexpr size_t bytes = sizeof(float) * (64 * NC + 16 * W1ROW) + 64 * (sizeof(double2) + sizeof(float2) +
                                                                                    sizeof(float));
};

// Work items come from the binning's queue; each chunk's samples (AdjRec, written
// by the binning with e^{i psi} and the TOD gradient) are staged by one thread each.
template <int CT, bool DET>
__global__ void __launch_bounds__(256)
k_scatter_mfma(const int4 *__restrict__ items, int *__restrict__ totals, const AdjRec *__restrict__ rec,
               const int *__restrict__ perm, float *__restrict__ gmaps, float *__restrict__ pg, int cols, int ncp,
               int ncomp, int nkc, double beta) {
    constexpr int NC = 16 * CT;
    extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte operands
    float *Vsh = (float *)smem_d;                // [64 samples][NC]
    float *W1 = Vsh + 64 * NC;                   // [16][W1ROW]: theta weights (rows 0-7), phi weights (8-15)
    double2 *E1 = (double2 *)(W1 + 16 * W1ROW);  // [64] e^{i psi} (64 NC + 1040 floats: 16-byte aligned)
    float2 *UV = (float2 *)(E1 + 64);            // [64] (u - floor u, v - floor v)
    float *Ys = (float *)(UV + 64);              // [64]
    __shared__ int item_sh;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, grp = lane >> 4;
    const int nitems = totals[1];
    const float nbl = -(float)beta * 1.44269504088896341f;  // -beta log2(e)
    // with many items (over ~64 per workgroup) they are taken in runs of consecutive
    // ones, one queue atomic per run (the single counter is contended otherwise)
    int run = nitems / (64 * (int)gridDim.x);
    run = run < 1 ? 1 : (run > 32 ? 32 : run);
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&totals[2], run);
        __syncthreads();
        const int i0 = __builtin_amdgcn_readfirstlane(item_sh);  // read before the first barrier below
        if (i0 >= nitems) break;
        const int iend = i0 + run < nitems ? i0 + run : nitems;
        for (int it = i0; it < iend; ++it) {
            const int4 item = items[it];
            const int row0 = item.x / nkc, col0 = item.x - (item.x / nkc) * nkc;
            floatx4 acc[CT];
    #pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int ch = 0; ch < item.z; ch += 64) {
                const int ns = item.z - ch < 64 ? item.z - ch : 64;
                if (tid < 64) {
                    double2 e1 = make_double2(1.0, 0.0);
                    float2 uv = make_float2(0.f, 0.f);
                    float yy = 0.f;
                    if (tid < ns) {
                        const int pos = DET ? perm[item.y + ch + tid] : item.y + ch + tid;
                        const AdjRec q = rec[pos];
                        e1 = make_double2(q.cps, q.sps);
                        uv = make_float2(q.fu, q.fv);
                        yy = q.y;
                    }
                    E1[tid] = e1;
                    UV[tid] = uv;
                    Ys[tid] = yy;
                }
                __syncthreads();
                for (int e = tid; e < 64 * 16; e += 256) {
                    const int q = e >> 6, sl = e & 63;
                    float w = 0.f;
                    if (sl < ns) {
                        const float2 uv = UV[sl];
                        w = es_weight_f32(((q < 8 ? uv.x : uv.y) + (float)(3 - (q & 7))) * 0.25f, nbl);
                    }
                    W1[q * W1ROW + sl] = w;
                }
                {
                    // V[s][c] = y_s basis_c(psi_s): 4 lanes per sample, NC/4 components each
                    const int sl = tid >> 2, qq = tid & 3;
                    constexpr int PER = NC / 4;
                    const int c0 = qq * PER;
                    const double2 e1 = E1[sl];
                    const float yy = Ys[sl];
                    int kc = c0 >> 1;  // PER is even: the range starts on a cos/sin pair
                    double2 z = cpow_int(e1, kc);
                    float *vrow = Vsh + sl * NC;
                    for (int j = 0; j < PER; ++j) {
                        const int c = c0 + j;
                        float vv = 0.f;
                        if (c < ncomp) {
                            if ((c >> 1) > kc) {
                                z = cmul(z, e1);
                                ++kc;
                            }
                            vv = yy * (float)((c & 1) ? z.y : z.x);
                        }
                        vrow[c] = vv;
                    }
                }
                __syncthreads();
                // PG[tap][c] += sum_s W[tap][s] V[s][c] with W[tap][s] = w_theta_s(tap / 8) w_phi_s(tap % 8)
                // formed from the 1-d weights as the operand is read; wave wv owns taps 16 wv .. 16 wv + 15
                const int tap = 16 * wv + r;
                const float *wth = W1 + (tap >> 3) * W1ROW + grp;  // A[i = tap r][k = sample grp]
                const float *wph = W1 + (8 + (tap & 7)) * W1ROW + grp;
                const float *vb = Vsh + grp * NC + r;               // B[k = sample grp][j = comp r]
    #pragma unroll 4
                for (int ks = 0; ks < 16; ++ks) {
                    const float a = wth[4 * ks] * wph[4 * ks];
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, vb[4 * ks * NC + 16 * ct], acc[ct], 0, 0, 0);
                }
                __syncthreads();
            }
            // D[i][j] in lane j + 16 (i/4), register i%4: tap 16 wv + 4 grp + v, component 16 ct + r
    #pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = 16 * wv + 4 * grp + v;
                if constexpr (DET) {
                    // the item's patch gradient, summed per pixel in a fixed order by k_scatter_reduce
                    float *dst = pg + ((size_t)it * 64 + t) * NC;
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct) dst[16 * ct + r] = acc[ct][v];
                } else {
                    float *base = gmaps + ((size_t)(row0 + (t >> 3)) * cols + (col0 + (t & 7))) * ncp;
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        const int c = 16 * ct + r;
                        if (c < ncomp && c != 1) atomic_add(base + c, acc[ct][v]);  // basis_1 = sin 0 = 0
                    }
                }
            }
        }
    }
}

// Split products (the default): the same patch gradients from
// v_mfma_f32_16x16x32_f16, to FP32 accuracy.  Operands are written as two FP16
// parts, x = hi + lo with hi = fp16(x), lo = fp16(x - hi) (|x - hi - lo| <= 2^-22 |x|),
// and PG ~ Wh Vh + Wh Vl + Wl Vh (the omitted Wl Vl is below 2^-22 of the product):
// three FP16 products per 16 x 16 x 32 block, 3/16 of the matrix time of the FP32
// form.  Ranges: tap weights (in [0, 1]) are scaled by 2^14, the chunk's V by
// 2^(14 - e) with 2^e above its largest |y|; each chunk's product goes to a
// temporary accumulator that is added, unscaled, into the item's sums.  The
// operand layout of the 16x16x32 instruction: A[i][k] in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; D as in the FP32 form.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

template <int CT>
struct SplitScatterLds {
    static constexpr size_t bytes = 2 * (2 * (size_t)CT * 64 * sizeof(half8)) + sizeof(float) * 16 * W1ROW +
                                    64 * (sizeof(double2) + sizeof(float2) + sizeof(float));
};

template <int CT, bool DET>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CT <= 5 ? 5 : 3)))
k_scatter_split(const int4 *__restrict__ items, int *__restrict__ totals, const AdjRec *__restrict__ rec,
                const int *__restrict__ perm, float *__restrict__ gmaps, float *__restrict__ pg, int cols, int ncp,
                int ncomp, int nkc, double beta) {
    constexpr int NC = 16 * CT;
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    half8 *Bhi = (half8 *)smem_d;                // [2 sample halves][CT][64 lanes]
    half8 *Blo = Bhi + 2 * CT * 64;
    float *W1 = (float *)(Blo + 2 * CT * 64);    // [16][W1ROW]: theta weights (rows 0-7), phi weights (8-15)
    double2 *E1 = (double2 *)(W1 + 16 * W1ROW);  // [64] e^{i psi} (1040 floats after 16-byte blocks: aligned)
    float2 *UV = (float2 *)(E1 + 64);            // [64] (u - floor u, v - floor v)
    float *Ys = (float *)(UV + 64);              // [64] y 2^(14 - e)
    __shared__ int item_sh;
    __shared__ float osc_sh;  // 2^(e - 28): undoes both scalings

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, grp = lane >> 4;
    const int nitems = totals[1];
    const float nbl = -(float)beta * 1.44269504088896341f;  // -beta log2(e)
    // with many items (over ~64 per workgroup) they are taken in runs of consecutive
    // ones, one queue atomic per run (the single counter is contended otherwise)
    int run = nitems / (64 * (int)gridDim.x);
    run = run < 1 ? 1 : (run > 32 ? 32 : run);
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&totals[2], run);
        __syncthreads();
        const int i0 = __builtin_amdgcn_readfirstlane(item_sh);  // read before the first barrier below
        if (i0 >= nitems) break;
        const int iend = i0 + run < nitems ? i0 + run : nitems;
        for (int it = i0; it < iend; ++it) {
            const int4 item = items[it];
            const int row0 = item.x / nkc, col0 = item.x - (item.x / nkc) * nkc;
            floatx4 acc[CT];
    #pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int ch = 0; ch < item.z; ch += 64) {
                const int ns = item.z - ch < 64 ? item.z - ch : 64;
                if (tid < 64) {  // one wave: one sample per lane
                    double2 e1 = make_double2(1.0, 0.0);
                    float2 uv = make_float2(0.f, 0.f);
                    float yy = 0.f;
                    if (tid < ns) {
                        const int pos = DET ? perm[item.y + ch + tid] : item.y + ch + tid;
                        const AdjRec q = rec[pos];
                        e1 = make_double2(q.cps, q.sps);
                        uv = make_float2(q.fu, q.fv);
                        yy = q.y;
                    }
                    float m = fabsf(yy);
    #pragma unroll
                    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
                    int e = 0;
                    if (m > 0.f) (void)frexpf(m, &e);  // m < 2^e
                    E1[tid] = e1;
                    UV[tid] = uv;
                    Ys[tid] = ldexpf(yy, 14 - e);  // exact
                    if (tid == 0) osc_sh = ldexpf(1.f, e - 28);
                }
                __syncthreads();
                for (int e = tid; e < 64 * 16; e += 256) {
                    const int q = e >> 6, sl = e & 63;
                    float w = 0.f;
                    if (sl < ns) {
                        const float2 uv = UV[sl];
                        w = es_weight_f32(((q < 8 ? uv.x : uv.y) + (float)(3 - (q & 7))) * 0.25f, nbl);
                    }
                    W1[q * W1ROW + sl] = w;
                }
                {
                    // V[s][c] = y_s basis_c(psi_s) (scaled), split and written in the B layout:
                    // sample s -> half s / 32, lane group (s % 32) / 8, element s % 8; component c ->
                    // tile c / 16, lane c % 16.  4 lanes per sample; lane qq takes the orders
                    // k = qq + 4 j (components 2k, 2k + 1: tile j / 2, lanes 2 qq + 8 (j % 2) and
                    // the next), so its offsets are compile-time after the base, and steps the
                    // phase by e^{4 i psi}.
                    const int sl = tid >> 2, qq = tid & 3;
                    const double2 e1 = E1[sl];
                    const double2 e2 = cmul(e1, e1), e4 = cmul(e2, e2);
                    double2 z = qq == 0 ? make_double2(1.0, 0.0) : qq == 1 ? e1 : qq == 2 ? e2 : cmul(e2, e1);
                    const float yy = Ys[sl];
                    const int base = ((sl >> 5) * CT * 64 + 16 * ((sl & 31) >> 3)) * 8 + (sl & 7) + 16 * qq;
                    _Float16 *bh = (_Float16 *)Bhi + base, *bl = (_Float16 *)Blo + base;
    #pragma unroll
                    for (int j = 0; j < 2 * CT; ++j) {
                        const int k = qq + 4 * j;
                        const float vc = 2 * k < ncomp ? yy * (float)z.x : 0.f;
                        const float vs = 2 * k + 1 < ncomp ? yy * (float)z.y : 0.f;
                        const int o = (j >> 1) * 512 + 64 * (j & 1);
                        const _Float16 hc = (_Float16)vc, hs = (_Float16)vs;
                        bh[o] = hc;
                        bl[o] = (_Float16)(vc - (float)hc);
                        bh[o + 8] = hs;
                        bl[o + 8] = (_Float16)(vs - (float)hs);
                        z = cmul(z, e4);
                    }
                }
                __syncthreads();
                {
                    // A: wave wv's taps 16 wv + r, samples 32 kh + 8 grp + q
                    const int tap = 16 * wv + r;
                    const float *wth = W1 + (tap >> 3) * W1ROW + 8 * grp;
                    const float *wph = W1 + (8 + (tap & 7)) * W1ROW + 8 * grp;
                    half8 ah[2], al[2];
    #pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
    #pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const float w = wth[32 * kh + q] * wph[32 * kh + q] * 16384.f;
                            const _Float16 h = (_Float16)w;
                            ah[kh][q] = h;
                            al[kh][q] = (_Float16)(w - (float)h);
                        }
                    const float osc = osc_sh;
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        floatx4 t = floatx4{0.f, 0.f, 0.f, 0.f};
    #pragma unroll
                        for (int kh = 0; kh < 2; ++kh) {
                            const half8 bh = Bhi[(kh * CT + ct) * 64 + lane], bl = Blo[(kh * CT + ct) * 64 + lane];
                            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[kh], bh, t, 0, 0, 0);
                            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kh], bl, t, 0, 0, 0);
                            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kh], bh, t, 0, 0, 0);
                        }
    #pragma unroll
                        for (int v = 0; v < 4; ++v) acc[ct][v] = fmaf(t[v], osc, acc[ct][v]);
                    }
                }
                __syncthreads();
            }
            // D[i][j] in lane j + 16 (i/4), register i%4: tap 16 wv + 4 grp + v, component 16 ct + r
    #pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = 16 * wv + 4 * grp + v;
                if constexpr (DET) {
                    // the item's patch gradient, summed per pixel in a fixed order by k_scatter_reduce
                    float *dst = pg + ((size_t)it * 64 + t) * NC;
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct) dst[16 * ct + r] = acc[ct][v];
                } else {
                    float *base = gmaps + ((size_t)(row0 + (t >> 3)) * cols + (col0 + (t & 7))) * ncp;
    #pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        const int c = 16 * ct + r;
                        if (c < ncomp && c != 1) atomic_add(base + c, acc[ct][v]);  // basis_1 = sin 0 = 0
                    }
                }
            }
        }
    }
}

// Deterministic mode, sample order.  The binning ranks the samples of an anchor in
// the order its atomics happen to run, so the same samples can land in different
// 64-sample chunks from run to run.  In this mode every anchor is one work item and
// this kernel sorts the item's samples by their index (a bitonic sort of (index,
// position) pairs in LDS, one workgroup per item of at most DET_MAXN samples), writing
// perm[first + i] = the sorted position of the i-th sample in index order; the scatter
// reads its records through perm.  It also records the largest item (totals[3]).
constexpr int DET_MAXN = 8192;

__global__ void __launch_bounds__(256)
k_det_order(const int4 *__restrict__ items, const int *__restrict__ totals, const AdjRec *__restrict__ rec,
            int *__restrict__ perm, int *__restrict__ maxn) {
    __shared__ unsigned key[DET_MAXN], val[DET_MAXN];
    const int it = blockIdx.x;
    if (it >= totals[1]) return;
    const int4 item = items[it];
    const int n = item.z, tid = threadIdx.x;
    if (tid == 0) atomicMax(maxn, n);
    if (n > DET_MAXN) return;  // the host splits the pass and bins again
    int np = 64;
    while (np < n) np <<= 1;
    for (int i = tid; i < np; i += 256) {
        key[i] = i < n ? (unsigned)rec[item.y + i].idx : 0xffffffffu;
        val[i] = (unsigned)(item.y + i);
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < np; i += 256) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const unsigned a = key[i], b = key[l];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[l] = a;
                        const unsigned t = val[i];
                        val[i] = val[l];
                        val[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < n; i += 256) perm[item.y + i] = (int)val[i];
}

// Deterministic mode: gmaps[R][C] += sum over the anchors (R - i, C - j), i, j < 8, in that
// order, and over each anchor's items in order, of the items' patch gradients at tap
// (i, j).  One workgroup per 8 x 8 pixel tile; the item ranges of the tile's 15 x 15
// anchors go to LDS first (an anchor's items are consecutive: ceil(count / chunk) of
// them from offs[key].y).  Thread (pixel, part) sums CT float4s of its pixel (the map
// record holds ncp <= 16 CT floats; the patch gradients 16 CT).
template <int CT>
__global__ void __launch_bounds__(256)
k_scatter_reduce(const float4 *__restrict__ pg, const int *__restrict__ count, const int2 *__restrict__ offs,
                 float *__restrict__ gmaps, int rows, int cols, int ncp, int nkr, int nkc, int chunk) {
    constexpr int NC4 = 4 * CT;  // float4s per tap
    __shared__ int2 rng[15 * 15];
    const int tiles_c = (cols + 7) / 8;
    const int R0 = 8 * (blockIdx.x / tiles_c), C0 = 8 * (blockIdx.x - (blockIdx.x / tiles_c) * tiles_c);
    const int tid = threadIdx.x;
    if (tid < 225) {
        const int ar = R0 - 7 + tid / 15, ac = C0 - 7 + tid % 15;
        int2 v = make_int2(0, 0);
        if (ar >= 0 && ar < nkr && ac >= 0 && ac < nkc) {
            const int64_t k = (int64_t)ar * nkc + ac;
            const int c = count[k];
            if (c > 0) v = make_int2(offs[k].y, (c + chunk - 1) / chunk);
        }
        rng[tid] = v;
    }
    __syncthreads();
    const int pix = tid >> 2, part = tid & 3;
    const int pr = pix >> 3, pc = pix & 7;
    const int R = R0 + pr, C = C0 + pc;
    if (R >= rows || C >= cols) return;
    float4 acc[CT];
#pragma unroll
    for (int q = 0; q < CT; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            const int2 g = rng[(pr + 7 - i) * 15 + (pc + 7 - j)];
            for (int it = g.x; it < g.x + g.y; ++it) {
                const float4 *src = pg + ((size_t)it * 64 + 8 * i + j) * NC4 + part * CT;
#pragma unroll
                for (int q = 0; q < CT; ++q) {
                    const float4 v = src[q];
                    acc[q].x += v.x;
                    acc[q].y += v.y;
                    acc[q].z += v.z;
                    acc[q].w += v.w;
                }
            }
        }
    float4 *dst = (float4 *)(gmaps + ((size_t)R * cols + C) * ncp) + part * CT;
#pragma unroll
    for (int q = 0; q < CT; ++q) {
        if (4 * (part * CT + q) >= ncp) break;  // CT may round the map's tile count up
        float4 o = dst[q];
        o.x += acc[q].x;
        o.y += acc[q].y;
        o.z += acc[q].z;
        o.w += acc[q].w;
        dst[q] = o;
    }
}

template <int CT>
hipError_t launch_scatter_split(sc_plan *p, void *gmaps) {
    const size_t lds = SplitScatterLds<CT>::bytes;
    auto kern = p->det_adjoint ? k_scatter_split<CT, true> : k_scatter_split<CT, false>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 256, lds, p->gather_wgs_per_cu);
    const BinGeom g = sc_bin_geom(p);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, p->stream, p->bw.items, p->bw.totals,
                       (const AdjRec *)p->bw.sorted.rec, p->bw.key, (float *)gmaps, p->pg, p->cols, p->ncp, p->ncomp,
                       g.nkc,
                       p->beta);
    return hipGetLastError();
}

template <int CT>
hipError_t launch_scatter_mfma(sc_plan *p, void *gmaps) {
    const size_t lds = ScatterLds<CT>::bytes;
    auto kern = p->det_adjoint ? k_scatter_mfma<CT, true> : k_scatter_mfma<CT, false>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 256, lds, p->gather_wgs_per_cu);
    const BinGeom g = sc_bin_geom(p);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, p->stream, p->bw.items, p->bw.totals,
                       (const AdjRec *)p->bw.sorted.rec, p->bw.key, (float *)gmaps, p->pg, p->cols, p->ncp, p->ncomp,
                       g.nkc,
                       p->beta);
    return hipGetLastError();
}

hipError_t launch_scatter_mfma_any(sc_plan *p, void *gmaps) {
    const int ct = (p->ncomp + 15) / 16;
    if (p->gather_mma == 1) {  // split FP16 products (the plan's product form, as for the gather)
        if (ct <= 1) return launch_scatter_split<1>(p, gmaps);
        if (ct <= 2) return launch_scatter_split<2>(p, gmaps);
        if (ct <= 3) return launch_scatter_split<3>(p, gmaps);
        if (ct <= 5) return launch_scatter_split<5>(p, gmaps);
        if (ct <= 9) return launch_scatter_split<9>(p, gmaps);
        if (ct <= 13) return launch_scatter_split<13>(p, gmaps);
        return launch_scatter_split<16>(p, gmaps);
    }
    if (ct <= 1) return launch_scatter_mfma<1>(p, gmaps);
    if (ct <= 2) return launch_scatter_mfma<2>(p, gmaps);
    if (ct <= 3) return launch_scatter_mfma<3>(p, gmaps);
    if (ct <= 5) return launch_scatter_mfma<5>(p, gmaps);
    if (ct <= 9) return launch_scatter_mfma<9>(p, gmaps);
    if (ct <= 13) return launch_scatter_mfma<13>(p, gmaps);
    return launch_scatter_mfma<16>(p, gmaps);
}

template <int CT>
hipError_t launch_reduce(sc_plan *p, void *gmaps) {
    const BinGeom g = sc_bin_geom(p);
    const int tiles = ((p->rows + 7) / 8) * ((p->cols + 7) / 8);
    hipLaunchKernelGGL(k_scatter_reduce<CT>, dim3(tiles), dim3(256), 0, p->stream, (const float4 *)p->pg,
                       p->bw.count, p->bw.offs, (float *)gmaps, p->rows, p->cols, p->ncp, g.nkr, g.nkc, p->bin_chunk);
    return hipGetLastError();
}

}  // namespace

bool sc_scatter_binned_supported(const sc_plan *p) {
    return p->prec != SC_FP64 && p->W == 8 && p->ncomp <= 256 && !p->gather_direct;
}

// Deterministic mode, after the binning (one item per anchor): the sample order of
// every item into the binning's key buffer (free after the binning), and the largest
// item into totals[3] (to be read back: above DET_MAXN the pass must be split).
hipError_t sc_launch_det_order(sc_plan *p, int nitems) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_order, dim3((unsigned)nitems), dim3(256), 0, p->stream, p->bw.items, p->bw.totals,
                       (const AdjRec *)p->bw.sorted.rec, p->bw.key, p->bw.totals + 3);
    return hipGetLastError();
}
int sc_det_max_items() { return DET_MAXN; }

// Deterministic mode, after the scatter of a pass has written its patch gradients (the
// reduction's tile count must match the scatter's: the same (ncomp + 15) / 16 rounding).
hipError_t sc_launch_scatter_reduce(sc_plan *p, void *gmaps) {
    const int ct = (p->ncomp + 15) / 16;
    if (ct <= 1) return launch_reduce<1>(p, gmaps);
    if (ct <= 2) return launch_reduce<2>(p, gmaps);
    if (ct <= 3) return launch_reduce<3>(p, gmaps);
    if (ct <= 5) return launch_reduce<5>(p, gmaps);
    if (ct <= 9) return launch_reduce<9>(p, gmaps);
    if (ct <= 13) return launch_reduce<13>(p, gmaps);
    return launch_reduce<16>(p, gmaps);
}

// Scatter of one pass (binned: binning with the pass's TOD gradient already done).
hipError_t sc_launch_scatter_binned(sc_plan *p, void *gmaps) { return launch_scatter_mfma_any(p, gmaps); }

hipError_t sc_launch_scatter(sc_plan *p, const double *ptg, int64_t n, const void *y, void *gmaps) {
    const double two_pi = 6.283185307179586477;
    const double inv_hth = (double)p->n2os / two_pi, inv_hph = (double)p->nphi / two_pi;
    int64_t nblk = (n + 3) / 4;
    if (nblk > 65536) nblk = 65536;
    if (p->prec == SC_FP64)
        hipLaunchKernelGGL(k_scatter_direct<double>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const double *)y, (double *)gmaps, p->cols, p->ncp, p->ncomp, p->W, p->beta, inv_hth,
                           inv_hph, p->n2os, p->nphi);
    else
        hipLaunchKernelGGL(k_scatter_direct<float>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const float *)y, (float *)gmaps, p->cols, p->ncp, p->ncomp, p->W, p->beta, inv_hth,
                           inv_hph, p->n2os, p->nphi);
    return hipGetLastError();
}
