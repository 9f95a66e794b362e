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

}  // namespace

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
