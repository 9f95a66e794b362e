// fft_lds.h -- mixed-radix (2, 3, 4, 5) Stockham autosort FFT of one complex
// FP64 sequence held in LDS, computed by one workgroup.
//
// Each stage of radix R reads R strided inputs per butterfly, applies the
// twiddles e^{DIR 2 pi i r (j mod Ns) / (Ns R)}, does a radix-R DFT in
// registers and writes the R outputs Ns apart; all reads of a stage finish
// (barrier) before its writes, so one LDS buffer suffices.  DIR = -1 is the
// forward transform sum_j x_j e^{-2 pi i n j / N}, DIR = +1 the unnormalised
// inverse.  Twiddles come from a table tw[t] = e^{-2 pi i t / N}.
#pragma once

#include "sc_common.h"

// Threads per transform workgroup and the longest transform each size handles
// (register staging holds ceil(MAXN / (R * NT)) radix-R butterflies per thread).
#define SC_FFT_NT 256
#define SC_FFT_NT_BIG 512
#define SC_FFT_MAXN_PER_THREAD 16

__device__ __forceinline__ double2 mul_i(double2 a, int dir) {
    // dir * i * a
    return dir > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <int R, int DIR>
__device__ __forceinline__ void dft_small(double2 *v);

template <>
__device__ __forceinline__ void dft_small<2, -1>(double2 *v) {
    double2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}
template <>
__device__ __forceinline__ void dft_small<2, 1>(double2 *v) {
    dft_small<2, -1>(v);
}

template <int DIR>
__device__ __forceinline__ void dft4(double2 *v) {
    double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    double2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    double2 id13 = mul_i(d13, DIR);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, id13);
    v[3] = csub(d02, id13);
}
template <>
__device__ __forceinline__ void dft_small<4, -1>(double2 *v) { dft4<-1>(v); }
template <>
__device__ __forceinline__ void dft_small<4, 1>(double2 *v) { dft4<1>(v); }

template <int DIR>
__device__ __forceinline__ void dft3(double2 *v) {
    const double s60 = 0.86602540378443864676;  // sin(2 pi / 3)
    double2 t1 = cadd(v[1], v[2]);
    double2 t2 = make_double2(v[0].x - 0.5 * t1.x, v[0].y - 0.5 * t1.y);
    double2 t3 = mul_i(cscale(csub(v[1], v[2]), s60), DIR);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
}
template <>
__device__ __forceinline__ void dft_small<3, -1>(double2 *v) { dft3<-1>(v); }
template <>
__device__ __forceinline__ void dft_small<3, 1>(double2 *v) { dft3<1>(v); }

template <int DIR>
__device__ __forceinline__ void dft5(double2 *v) {
    const double c1 = 0.30901699437494742410;   // cos(2 pi / 5)
    const double c2 = -0.80901699437494742410;  // cos(4 pi / 5)
    const double s1 = 0.95105651629515357212;   // sin(2 pi / 5)
    const double s2 = 0.58778525229247312917;   // sin(4 pi / 5)
    double2 t1 = cadd(v[1], v[4]), t3 = csub(v[1], v[4]);
    double2 t2 = cadd(v[2], v[3]), t4 = csub(v[2], v[3]);
    double2 b1 = make_double2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    double2 b2 = make_double2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    double2 e1 = make_double2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    double2 e2 = make_double2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    double2 ie1 = mul_i(e1, DIR), ie2 = mul_i(e2, DIR);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, ie1);
    v[4] = csub(b1, ie1);
    v[2] = cadd(b2, ie2);
    v[3] = csub(b2, ie2);
}
template <>
__device__ __forceinline__ void dft_small<5, -1>(double2 *v) { dft5<-1>(v); }
template <>
__device__ __forceinline__ void dft_small<5, 1>(double2 *v) { dft5<1>(v); }

template <int R, int DIR, int NT>
__device__ __forceinline__ void stockham_stage(double2 *buf, int N, int Ns, const double2 *__restrict__ tw,
                                               int tid, int nth) {
    constexpr int B = (SC_FFT_MAXN_PER_THREAD * NT / R + NT - 1) / NT;
    const int nb = N / R;
    const int twstep = N / (Ns * R);
    double2 v[B][R];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * nth;
        if (j < nb) {
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[j + r * nb];
                if (r > 0) {
                    double2 w = tw[r * k * twstep];
                    if (DIR > 0) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[b][r] = x;
            }
            dft_small<R, DIR>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * nth;
        if (j < nb) {
            const int k = j % Ns;
            const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[idx + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

// In-place transform of buf[0 .. P.n) (LDS) by NT threads; requires
// P.n <= SC_FFT_MAXN_PER_THREAD * NT.  Starts and ends with a barrier-complete buffer.
template <int DIR, int NT>
__device__ void fft_lds(double2 *buf, const FftPlan &P, const double2 *__restrict__ tw, int tid, int nth) {
    int Ns = 1;
    for (int s = 0; s < P.nst; ++s) {
        const int R = P.r[s];
        if (R == 4)
            stockham_stage<4, DIR, NT>(buf, P.n, Ns, tw, tid, nth);
        else if (R == 2)
            stockham_stage<2, DIR, NT>(buf, P.n, Ns, tw, tid, nth);
        else if (R == 3)
            stockham_stage<3, DIR, NT>(buf, P.n, Ns, tw, tid, nth);
        else
            stockham_stage<5, DIR, NT>(buf, P.n, Ns, tw, tid, nth);
        Ns *= R;
    }
}
