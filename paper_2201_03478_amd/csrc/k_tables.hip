// k_tables.hip -- constant tables of a plan, computed on the device.
//
//  * FFT twiddles e^{-2 pi i t / N} for the three transform lengths.
//  * Gauss-Legendre nodes on [-1, 1] (Newton iteration on P_n).
//  * Deconvolution factors of the exponential-of-semicircle interpolation
//    kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1, of width W cells:
//    for grid spacing h the interpolant reproduces e^{i n x} times
//        hhat(n) = (W/2) int_{-1}^{1} phi(z) cos(n z W h / 2) dz,
//    computed with z = sin t (which removes the endpoint square root) by
//    Gauss-Legendre quadrature in t.  Each spectral coefficient is divided by
//    hhat (theta and phi factors) before the grid is synthesised.
//  * sqrt((l+1)^2 - x^2) and its reciprocal for 0 <= x, l <= lmax (the roots of
//    the recursion coefficients).
//  * sqrt(C(2 l, l + n)) as (mantissa, binary exponent) pairs: the prefactor of
//    the closed-form start values d^l_{l k} and d^l_{m l} of the Wigner-d
//    recursion (Wigner's explicit sum with a single surviving term).
#include "sc_common.h"

namespace {

// Pass-major twiddles of a plan: pass s (span NS = ns[s], radix R, twiddle step
// tws[s]) holds e^{-2 pi i r k tws / N} for r = 1 .. R-1, k = 0 .. NS-1 at
// (NS - 1) + (r - 1) NS + k, so the lanes of a pass (consecutive k) read
// consecutive entries.  The passes' blocks fill [0, N - 1) exactly (their sizes
// (R - 1) NS telescope to N - 1).
__global__ void k_pass_twiddles(double2 *tw, FftPlan P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.n) return;
    double2 v = make_double2(1.0, 0.0);
    for (int s = 0; s < P.nst; ++s) {
        const int NS = P.ns[s], R = P.r[s];
        const int local = e - (NS - 1);
        if (local >= 0 && local < (R - 1) * NS) {
            const int r = 1 + local / NS, k = local - (r - 1) * NS;
            const long long t = (long long)r * k * P.tws[s];
            double sn, cs;
            sincospi(-2.0 * (double)t / (double)P.n, &sn, &cs);
            v = make_double2(cs, sn);
        }
    }
    tw[e] = v;
}

__global__ void k_gauss_legendre(double *x, double *w, int nq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    double z = cospi((i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int j = 1; j < nq; ++j) {
            double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
            p0 = p1;
            p1 = p2;
        }
        dp = nq * (z * p1 - p0) / (z * z - 1.0);
        double dz = p1 / dp;
        z -= dz;
        if (fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int j = 1; j < nq; ++j) {
        double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
    }
    dp = nq * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
}

// hhat(n) for the kernel on a grid of spacing h (see header comment).
__device__ double kernel_transform(double n, double h, int W, double beta, const double *glx, const double *glw,
                                   int nq) {
    double acc = 0.0;
    const double half_pi = 1.5707963267948966192;
    for (int q = 0; q < nq; ++q) {
        const double t = half_pi * glx[q];
        double st, ct;
        sincos(t, &st, &ct);
        acc += glw[q] * exp(beta * (ct - 1.0)) * ct * cos(n * st * (double)W * h * 0.5);
    }
    return 0.5 * (double)W * half_pi * acc;
}

__global__ void k_deconv(double2 *phase, double *dphi, int lmax, int n2, int n2os, int nphi, int W,
                         double beta, const double *glx, const double *glw, int nq) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double two_pi = 6.283185307179586477;
    if (t < 2 * lmax + 1) {
        const int n = t - lmax;
        const double hh = kernel_transform((double)(n < 0 ? -n : n), two_pi / n2os, W, beta, glx, glw, nq);
        double s, c;
        sincospi(-(double)n / (double)n2, &s, &c);  // e^{-i n (pi / n2)}: half-ring shift
        const double f = 1.0 / ((double)n2 * hh);
        phase[t] = make_double2(c * f, s * f);
    }
    if (t <= lmax) dphi[t] = 1.0 / kernel_transform((double)t, two_pi / nphi, W, beta, glx, glw, nq);
}

// psi deconvolution: 1 / hhat(k) for the kernel on the npsi-point psi grid.
__global__ void k_psi_deconv(double *gpsi, int kmax, int npsi, int W, double beta, const double *glx,
                             const double *glw, int nq) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= kmax) gpsi[k] = 1.0 / kernel_transform((double)k, 6.283185307179586477 / npsi, W, beta, glx, glw, nq);
}

// Recursion roots: at [x][l], sqrt((l+1)^2 - x^2) and its reciprocal (zero where
// l + 1 <= x), so that the recursion coefficients of step l need one division.
__global__ void k_rec_roots(double2 *t, int lmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nl = lmax + 1;
    if (i >= nl * nl) return;
    const int x = (int)(i / nl), l = (int)(i - (int64_t)x * nl);
    const double v = (double)(l + 1) * (l + 1) - (double)x * x;  // exact
    double2 r = make_double2(0.0, 0.0);
    if (v > 0.0) {
        const double s = sqrt(v);
        r = make_double2(s, 1.0 / s);
    }
    t[i] = r;
}

__global__ void k_sqrt_binom(double *sm, int *se, int lmax, int kmax) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = id / (kmax + 1), n = id - l * (kmax + 1);
    if (l > lmax) return;
    double m = 0.5;
    int e = 1;  // 1.0
    if (n <= l) {
        // C(2l, l+n) = prod_{i=1}^{l-n} (l + n + i) / i
        for (int i = 1; i <= l - n; ++i) {
            int ee;
            m = frexp(m * ((double)(l + n + i) / (double)i), &ee);
            e += ee;
        }
        if (e & 1) {
            m *= 2.0;
            e -= 1;
        }
        m = sqrt(m);  // m in [0.5, 2): sqrt keeps it normal
        e /= 2;
        int ee;
        m = frexp(m, &ee);
        e += ee;
    } else {
        m = 0.0;
        e = 0;
    }
    sm[id] = m;
    se[id] = e;
}

}  // namespace

hipError_t sc_launch_tables(sc_plan *p) {
    const int bs = 256;
    // (sub-)transform lengths: the full lengths unless a transform is split
    hipLaunchKernelGGL(k_pass_twiddles, dim3((p->p2.n + bs - 1) / bs), dim3(bs), 0, p->stream, p->tw2, p->p2);
    hipLaunchKernelGGL(k_pass_twiddles, dim3((p->p2os.n + bs - 1) / bs), dim3(bs), 0, p->stream, p->tw2os, p->p2os);
    hipLaunchKernelGGL(k_pass_twiddles, dim3((p->pphi.n + bs - 1) / bs), dim3(bs), 0, p->stream, p->twphi, p->pphi);
    hipLaunchKernelGGL(k_gauss_legendre, dim3((p->nq + 63) / 64), dim3(64), 0, p->stream, p->glx, p->glw, p->nq);
    const int nt = 2 * p->lmax + 1;
    hipLaunchKernelGGL(k_deconv, dim3((nt + 63) / 64), dim3(64), 0, p->stream, p->phase, p->dphi, p->lmax, p->n2,
                       p->n2os, p->nphi, p->W, p->beta, p->glx, p->glw, p->nq);
    const int nb = (p->lmax + 1) * (p->kmax + 1);
    const int64_t nr = (int64_t)(p->lmax + 1) * (p->lmax + 1);
    hipLaunchKernelGGL(k_rec_roots, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, p->stream, p->rroot, p->lmax);
    hipLaunchKernelGGL(k_sqrt_binom, dim3((nb + 255) / 256), dim3(256), 0, p->stream, p->sbin_m, p->sbin_e,
                       p->lmax, p->kmax);
    return hipGetLastError();
}

hipError_t sc_launch_psi_tables(sc_plan *p) {
    const int bs = 256;
    hipLaunchKernelGGL(k_pass_twiddles, dim3((p->npsi + bs - 1) / bs), dim3(bs), 0, p->stream, p->twpsi, p->ppsi);
    hipLaunchKernelGGL(k_psi_deconv, dim3((p->kmax + 64) / 64), dim3(64), 0, p->stream, p->gpsi, p->kmax, p->npsi,
                       p->W, p->beta, p->glx, p->glw, p->nq);
    return hipGetLastError();
}
