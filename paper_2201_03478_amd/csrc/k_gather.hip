// k_gather.hip -- interpolation of the component maps and the per-sample k-sum.
//
// For a pointing (theta, phi, psi) the convolution is (Galloway et al. 2022,
// Sec. 2.1, Eq. 8 with the finite-resolution maps and interpolation described
// after the two-step algorithm)
//     c = sum_{i,j < W} w_theta(i) w_phi(j) sum_c basis_c(psi) M_c[r0 + i][q0 + j],
//     basis = (1, cos psi, sin psi, cos 2 psi, sin 2 psi, ...),
// with exponential-of-semicircle weights w(z) = exp(beta (sqrt(1 - z^2) - 1)),
// z = (x - x_node) / (W/2) in grid units.  The grid indices and the fractional
// offsets are formed in FP64 (a float phi near 2 pi would misplace the stencil
// by up to 2.4e-7 rad); psi is reduced in FP64 before its multiples are taken.
//
// v1 layout: one wave per sample, lanes over components.
#include "sc_common.h"

namespace {

template <typename T>
__device__ __forceinline__ T es_weight(T z, T beta) {
    const T q = (T)1 - z * z;
    return q > (T)0 ? exp(beta * (sqrt(q) - (T)1)) : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gather_v1(const double *__restrict__ ptg, int64_t n, const T *__restrict__ maps, T *__restrict__ tod, int cols,
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
        if (!(v < (double)nphi)) v = 0.0;  // 2 pi rounding, NaN
        if (v < 0.0) v = 0.0;
        const int q0 = (int)floor(v) - half + 1;
        T w = (T)0;
        if (lane < W)
            w = es_weight<T>((T)((u - (double)(r0 + lane)) / half), (T)beta);
        else if (lane < 2 * W)
            w = es_weight<T>((T)((v - (double)(q0 + lane - W)) / half), (T)beta);

        T acc[4] = {(T)0, (T)0, (T)0, (T)0};
        const int row0 = r0 + half - 1, col0 = q0 + half - 1;
        for (int i = 0; i < W; ++i) {
            const T wi = __shfl(w, i);
            for (int j = 0; j < W; ++j) {
                const T wij = wi * __shfl(w, W + j);
                const T *base = maps + ((size_t)(row0 + i) * cols + (col0 + j)) * ncp;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = lane + 64 * t;
                    if (c < ncomp) acc[t] += wij * base[c];
                }
            }
        }
        double psr = ps - two_pi * floor(ps / two_pi);
        T part = (T)0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = lane + 64 * t;
            if (c < ncomp) {
                T bas = (T)1;
                if (c > 0) {
                    const int kk = (c + 1) >> 1;
                    double sn, cs;
                    sincos((double)kk * psr, &sn, &cs);
                    bas = (T)((c & 1) ? cs : sn);
                }
                part += bas * acc[t];
            }
        }
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
        if (lane == 0) tod[s] = part;
    }
}

// ---------------------------------------------------------------------------
// Binned gather (W = 8).  A persistent workgroup takes work items from a queue;
// an item is up to BIN_CHUNK samples that share the stencil anchor (row0, col0)
// (see k_bin.hip).  The 8 x 8 x ncomp map block of the anchor is staged in LDS
// once; the samples are processed 64 at a time as a register-blocked product
//     X[s][c] = sum_{t < 64} w_s(t) P[t][c]      (w_s(t) = w_theta(i) w_phi(j))
// with each lane holding 4 samples x CPT components, followed by the k-sum
// sum_c basis_c(psi_s) X[s][c] and a reduction over the 16 lanes that hold the
// components of a sample.  cos k psi / sin k psi are formed in FP64: one
// sincos per lane and sample at the lane's first k, then rotations by e^{i psi}.
template <typename T, int CPT>
__global__ void __launch_bounds__(256)
k_gather_binned(const int4 *__restrict__ items, int *__restrict__ totals, BinSorted srt,
                const T *__restrict__ maps, T *__restrict__ tod, int cols, int ncp, int ncomp, int nkc,
                double beta) {
    constexpr int NC = 16 * CPT;  // staged components (zero-padded)
    extern __shared__ double smem_d[];
    T *Psh = (T *)smem_d;       // [64 taps][NC]
    T *Wsh = Psh + 64 * NC;     // [64 taps][64 samples]
    T *W1 = Wsh + 64 * 64;      // [64 samples][16]: 8 theta then 8 phi weights
    double *Psi = (double *)(W1 + 64 * 16);  // [64]
    double2 *E1 = (double2 *)(Psi + 64);     // [64] (cos psi, sin psi)
    int *Idx = (int *)(E1 + 64);             // [64]
    __shared__ int item_sh;

    const int tid = threadIdx.x;
    const int sg = tid >> 4, cg = tid & 15;
    const int nitems = totals[1];
    const T tbeta = (T)beta;
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&totals[2], 1);
        __syncthreads();
        const int it = item_sh;
        if (it >= nitems) break;
        const int4 item = items[it];
        const int row0 = item.x / nkc, col0 = item.x - (item.x / nkc) * nkc;
        for (int e = tid; e < 64 * NC; e += 256) {
            const int t = e / NC, c = e - t * NC;
            T v = (T)0;
            if (c < ncp) v = maps[((size_t)(row0 + (t >> 3)) * cols + (col0 + (t & 7))) * ncp + c];
            Psh[e] = v;
        }
        for (int ch = 0; ch < item.z; ch += 64) {
            const int ns = item.z - ch < 64 ? item.z - ch : 64;
            const int pos0 = item.y + ch;
            for (int e = tid; e < 64 * 16; e += 256) {
                const int sl = e >> 4, q = e & 15;
                T w = (T)0;
                if (sl < ns) {
                    const T f = (q < 8) ? (T)srt.fu[pos0 + sl] : (T)srt.fv[pos0 + sl];
                    const T z = (f + (T)(3 - (q & 7))) * (T)0.25;  // (x - node) / (W/2)
                    w = es_weight<T>(z, tbeta);
                }
                W1[e] = w;
            }
            if (tid < 64) {
                double ps = 0.0;
                int ix = -1;
                if (tid < ns) {
                    ps = srt.psi[pos0 + tid];
                    ix = srt.idx[pos0 + tid];
                }
                double sn, cs;
                sincos(ps, &sn, &cs);
                Psi[tid] = ps;
                E1[tid] = make_double2(cs, sn);
                Idx[tid] = ix;
            }
            __syncthreads();
            for (int e = tid; e < 64 * 64; e += 256) {
                const int t = e >> 6, sl = e & 63;
                Wsh[e] = W1[sl * 16 + (t >> 3)] * W1[sl * 16 + 8 + (t & 7)];
            }
            __syncthreads();

            T acc[4][CPT];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < CPT; ++c) acc[q][c] = (T)0;
#pragma unroll 4
            for (int t = 0; t < 64; ++t) {
                const T *wr = Wsh + t * 64 + 4 * sg;
                const T w0 = wr[0], w1 = wr[1], w2 = wr[2], w3 = wr[3];
                const T *pr = Psh + t * NC + cg * CPT;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const T pv = pr[c];
                    acc[0][c] = fma(w0, pv, acc[0][c]);
                    acc[1][c] = fma(w1, pv, acc[1][c]);
                    acc[2][c] = fma(w2, pv, acc[2][c]);
                    acc[3][c] = fma(w3, pv, acc[3][c]);
                }
            }

            const int c0 = cg * CPT;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int sl = 4 * sg + q;
                const double ps = Psi[sl];
                const double2 e1 = E1[sl];
                int k = (c0 + 1) >> 1;
                double sn, cs;
                sincos((double)k * ps, &sn, &cs);
                T part = (T)0;
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    const int c = c0 + j;
                    if (c < ncomp) {
                        if (c == 0) {
                            part += acc[q][j];
                        } else {
                            if (((c + 1) >> 1) > k) {
                                const double cn = cs * e1.x - sn * e1.y;
                                sn = sn * e1.x + cs * e1.y;
                                cs = cn;
                                ++k;
                            }
                            part = fma((T)((c & 1) ? cs : sn), acc[q][j], part);
                        }
                    }
                }
                part += __shfl_xor(part, 8);
                part += __shfl_xor(part, 4);
                part += __shfl_xor(part, 2);
                part += __shfl_xor(part, 1);
                if (cg == 0 && sl < ns) tod[Idx[sl]] = part;
            }
            __syncthreads();
        }
    }
}

template <typename T, int CPT>
hipError_t launch_binned(sc_plan *p, void *tod) {
    constexpr int NC = 16 * CPT;
    const size_t lds = sizeof(T) * (64 * NC + 64 * 64 + 64 * 16) + 64 * (sizeof(double) + sizeof(double2) + sizeof(int));
    auto kern = k_gather_binned<T, CPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu < 1) ncu = 256;
    const BinGeom g = sc_bin_geom(p);
    hipLaunchKernelGGL(kern, dim3(per_cu * ncu), dim3(256), lds, p->stream, p->bw.items, p->bw.totals,
                       p->bw.sorted, (const T *)p->maps, (T *)tod, p->cols, p->ncp, p->ncomp, g.nkc, p->beta);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_binned_t(sc_plan *p, void *tod) {
    const int cpt = (p->ncomp + 15) / 16;
    if (cpt <= 1) return launch_binned<T, 1>(p, tod);
    if (cpt <= 2) return launch_binned<T, 2>(p, tod);
    if (cpt <= 3) return launch_binned<T, 3>(p, tod);
    if (cpt <= 5) return launch_binned<T, 5>(p, tod);
    if (cpt <= 9) return launch_binned<T, 9>(p, tod);
    if (cpt <= 13) return launch_binned<T, 13>(p, tod);
    return launch_binned<T, 16>(p, tod);
}

}  // namespace

// W = 8 only; the FP64 staging of 208+ components would exceed the 160 KiB of LDS.
bool sc_gather_binned_supported(const sc_plan *p) {
    return p->W == 8 && p->ncomp <= (p->prec == SC_FP64 ? 208 : 256);
}

hipError_t sc_launch_gather_binned(sc_plan *p, void *tod) {
    if (p->prec == SC_FP64) return launch_binned_t<double>(p, tod);
    return launch_binned_t<float>(p, tod);
}

hipError_t sc_launch_gather(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    const double two_pi = 6.283185307179586477;
    const double inv_hth = (double)p->n2os / two_pi, inv_hph = (double)p->nphi / two_pi;
    int64_t nblk = (n + 3) / 4;
    if (nblk > 65536) nblk = 65536;
    if (p->prec == SC_FP64)
        hipLaunchKernelGGL(k_gather_v1<double>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const double *)p->maps, (double *)tod, p->cols, p->ncp, p->ncomp, p->W, p->beta,
                           inv_hth, inv_hph, p->n2os, p->nphi);
    else
        hipLaunchKernelGGL(k_gather_v1<float>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const float *)p->maps, (float *)tod, p->cols, p->ncp, p->ncomp, p->W, p->beta,
                           inv_hth, inv_hph, p->n2os, p->nphi);
    return hipGetLastError();
}
