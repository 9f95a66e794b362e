// fft_lds.h -- mixed-radix Stockham autosort FFT of one complex FP64 sequence
// held in LDS, computed by one workgroup.
//
// A transform of length N = 2^a 3^b 5^c is split into passes of radix
// R in {2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16}.  A pass of radix R reads R
// inputs N / R apart per butterfly, applies the twiddles
// e^{DIR 2 pi i r (j mod Ns) / (Ns R)}, does the R-point DFT in registers and
// writes the R outputs Ns apart (Ns = product of the earlier radices); all
// reads of a pass finish (barrier) before its writes, so one LDS buffer
// suffices.  Radices above 5 are register sub-transforms R = R1 R2 (R2 DFTs of
// length R1, constant twiddles e^{DIR 2 pi i n2 k1 / R}, R1 DFTs of length R2),
// so the data crosses LDS once per pass, not once per prime factor.
// DIR = -1 is the forward transform sum_j x_j e^{-2 pi i n j / N}, DIR = +1 the
// unnormalised inverse.  Pass twiddles come from a pass-major table: the pass
// with span Ns and twiddle step ts = N / (Ns R) finds e^{-2 pi i r k ts / N} at
// (Ns - 1) + (r - 1) Ns + k, so a wave's lanes (consecutive k) read one
// contiguous run; the first pass (Ns = 1) has unit twiddles and loads none.
//
// Size classes: NT threads per workgroup and at most PT points per thread
// (N <= NT PT); a radix-R pass holds ceil(PT / R) butterflies per thread.
#pragma once

#include "sc_common.h"

#define SC_FFT_NT 256
#define SC_FFT_NT_BIG 512
#define SC_FFT_PT 9
#define SC_FFT_NT_HUGE 1024
#define SC_FFT_PT_HUGE 9

// ---------------------------------------------------------------------------
// Compile-time cos / sin of 2 pi a / R (constants of the register sub-transforms):
// reduce to an octant, then Taylor series on |x| <= pi / 4.
namespace fftc {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double sin_small(double x) {
    double t = x, s = x;
    for (int n = 1; n <= 12; ++n) {
        t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        s += t;
    }
    return s;
}

constexpr double cos_small(double x) {
    double t = 1.0, s = 1.0;
    for (int n = 1; n <= 12; ++n) {
        t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        s += t;
    }
    return s;
}

struct CS {
    double c, s;
};

// cos and sin of the angle q pi / 2 + phi
constexpr CS quadrant(int q, double cphi, double sphi) {
    q &= 3;
    return q == 0 ? CS{cphi, sphi} : q == 1 ? CS{-sphi, cphi} : q == 2 ? CS{-cphi, -sphi} : CS{sphi, -cphi};
}

// e^{2 pi i a / R} = (cos, sin)
constexpr CS cis(int a, int R) {
    const int f = ((a % R) + R) % R;  // angle (pi / 4) * (8 f / R)
    const int u = 8 * f, o = u / R, rem = u - o * R;
    if ((o & 1) == 0) {
        const double x = (kPi / 4.0) * rem / R;  // angle = (o / 2) pi / 2 + x
        return quadrant(o / 2, cos_small(x), sin_small(x));
    }
    const double y = (kPi / 4.0) * (R - rem) / R;  // angle = (o / 2 + 1) pi / 2 - y
    return quadrant(o / 2 + 1, cos_small(y), -sin_small(y));
}

template <int R>
struct CisTable {
    double c[R], s[R];
    constexpr CisTable() : c(), s() {
        for (int a = 0; a < R; ++a) {
            const CS w = cis(a, R);
            c[a] = w.c;
            s[a] = w.s;
        }
    }
};

}  // namespace fftc

__device__ __forceinline__ double2 mul_i(double2 a, int dir) {
    // dir * i * a
    return dir > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Base DFTs (R = 2, 3, 4, 5), in place: v[k] <- sum_n v[n] e^{DIR 2 pi i n k / R}.

template <int DIR>
__device__ __forceinline__ void dft2(double2 *v) {
    const double2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
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

template <int R, int DIR>
__device__ __forceinline__ void dft_base(double2 *v) {
    if constexpr (R == 2)
        dft2<DIR>(v);
    else if constexpr (R == 3)
        dft3<DIR>(v);
    else if constexpr (R == 4)
        dft4<DIR>(v);
    else
        dft5<DIR>(v);
}

// x * e^{DIR 2 pi i e / R} for a twiddle exponent e that is a constant after unrolling;
// the trivial angles cost no multiplications.
template <int R, int DIR>
__device__ __forceinline__ double2 twiddle_const(double2 x, int e) {
    constexpr fftc::CisTable<R> T{};
    e %= R;
    if (e == 0) return x;
    if (2 * e == R) return make_double2(-x.x, -x.y);
    if (4 * e == R) return mul_i(x, DIR);
    if (4 * e == 3 * R) return mul_i(x, -DIR);
    return cmul(x, make_double2(T.c[e], DIR * T.s[e]));
}

// Composite DFT R = R1 R2 (Cooley-Tukey, all indices compile-time after unrolling):
// X[k1 + R1 k2] = sum_{n2} e^{DIR 2 pi i n2 k2 / R2} e^{DIR 2 pi i n2 k1 / R}
//                 sum_{n1} v[R2 n1 + n2] e^{DIR 2 pi i n1 k1 / R1}.
template <int R1, int R2, int DIR>
__device__ __forceinline__ void dft_ct(double2 *v) {
    constexpr int R = R1 * R2;
    double2 y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        double2 t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
        dft_base<R1, DIR>(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = twiddle_const<R, DIR>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        double2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2 * R1 + k1];
        dft_base<R2, DIR>(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft_small(double2 *v) {
    if constexpr (R <= 5)
        dft_base<R, DIR>(v);
    else if constexpr (R == 6)
        dft_ct<2, 3, DIR>(v);
    else if constexpr (R == 8)
        dft_ct<4, 2, DIR>(v);
    else if constexpr (R == 9)
        dft_ct<3, 3, DIR>(v);
    else if constexpr (R == 10)
        dft_ct<2, 5, DIR>(v);
    else if constexpr (R == 12)
        dft_ct<4, 3, DIR>(v);
    else if constexpr (R == 15)
        dft_ct<3, 5, DIR>(v);
    else
        dft_ct<4, 4, DIR>(v);  // 16
}

// ---------------------------------------------------------------------------
// One Stockham pass of radix R.

template <int R, int DIR, int NT, int PT>
__device__ __forceinline__ void stockham_stage(double2 *buf, int N, int Ns, unsigned mag,
                                               const double2 *__restrict__ tw, int tid, int nth) {
    constexpr int B = (PT + R - 1) / R;  // butterflies per thread: B NT >= N / R since N <= NT PT
    const int nb = N / R;
    double2 v[B][R];
    int widx[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * nth;
        if (j < nb) {
            // j = g Ns + k; the multiply-high is exact for j, Ns < 2^16
            const int g = Ns > 1 ? (int)__umulhi((unsigned)j, mag) : j;
            const int k = j - g * Ns;
            widx[b] = g * Ns * R + k;
            const double2 *twk = tw + (Ns - 1) + k;  // pass-major table: entry (r - 1) Ns
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[j + r * nb];
                if (r > 0 && Ns > 1) {
                    double2 w = twk[(r - 1) * Ns];
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
#pragma unroll
            for (int r = 0; r < R; ++r) buf[widx[b] + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

// In-place transform of buf[0 .. P.n) (LDS) by NT threads; requires P.n <= NT PT.
// Starts and ends with a barrier-complete buffer.
template <int DIR, int NT, int PT>
__device__ void fft_lds(double2 *buf, const FftPlan &P, const double2 *__restrict__ tw, int tid, int nth) {
    for (int s = 0; s < P.nst; ++s) {
        const int R = P.r[s], Ns = P.ns[s];
        const unsigned mg = P.mag[s];
        switch (R) {
            case 2: stockham_stage<2, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 3: stockham_stage<3, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 4: stockham_stage<4, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 5: stockham_stage<5, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 6: stockham_stage<6, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 8: stockham_stage<8, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 9: stockham_stage<9, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 10: stockham_stage<10, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 12: stockham_stage<12, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            case 15: stockham_stage<15, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
            default: stockham_stage<16, DIR, NT, PT>(buf, P.n, Ns, mg, tw, tid, nth); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Transforms whose length and radix sequence are compile-time constants: the
// same Stockham passes with every span, stride and twiddle step folded, one code
// path per pass (no runtime radix switch), so a kernel holds only its own passes.
// FftSpec<N, R0, R1, ...> lists the radices in pass order; FftGeneric selects the
// runtime-planned fft_lds.

template <int N, int... Rs>
struct FftSpec {};
struct FftGeneric {};

template <int R, int DIR, int NT, int N, int NS>
__device__ __forceinline__ void stockham_stage_c(double2 *buf, const double2 *__restrict__ tw, int tid) {
    constexpr int nb = N / R;
    constexpr int B = (nb + NT - 1) / NT;
    double2 v[B][R];
    int widx[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * NT;
        if ((b + 1) * NT <= nb || j < nb) {
            const int g = j / NS, k = j - g * NS;
            widx[b] = g * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[j + r * nb];
                if (NS > 1 && r > 0) {
                    double2 w = tw[(NS - 1) + (r - 1) * NS + k];  // pass-major table
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
        const int j = tid + b * NT;
        if ((b + 1) * NT <= nb || j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[widx[b] + r * NS] = v[b][r];
        }
    }
    __syncthreads();
}

template <int DIR, int NT, int N, int NS, int R, int... Rest>
__device__ __forceinline__ void fft_passes_c(double2 *buf, const double2 *__restrict__ tw, int tid) {
    stockham_stage_c<R, DIR, NT, N, NS>(buf, tw, tid);
    if constexpr (sizeof...(Rest) > 0) fft_passes_c<DIR, NT, N, NS * R, Rest...>(buf, tw, tid);
}

// The same passes with the twiddles taken from LDS: per pass with a span NS > 1
// only the base row w^k = e^{-2 pi i k / (R NS)}, k < NS (NS values), is stored,
// and w^{r k} is formed by repeated multiplication (r < 16 products: a relative
// error of a few 1e-16), so a transform needs no global loads once the bases of all
// its passes are in LDS.  The buffer holds complex128 or complex64 values (BT); the
// arithmetic is FP64 either way, so complex64 only rounds each pass's outputs.
template <int R, int DIR, int NT, int N, int NS, typename BT>
__device__ __forceinline__ void stockham_stage_l(BT *buf, const double2 *twl, int tid) {
    constexpr int nb = N / R;
    constexpr int B = (nb + NT - 1) / NT;
    double2 v[B][R];
    int widx[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * NT;
        if ((b + 1) * NT <= nb || j < nb) {
            const int g = j / NS, k = j - g * NS;
            widx[b] = g * NS * R + k;
            double2 w1 = make_double2(1.0, 0.0), w = w1;
            if (NS > 1) {
                w1 = twl[k];
                if (DIR > 0) w1.y = -w1.y;
                w = w1;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = ld2(buf + j + r * nb);
                if (NS > 1 && r > 0) {
                    x = cmul(x, w);
                    if (r + 1 < R) w = cmul(w, w1);
                }
                v[b][r] = x;
            }
            dft_small<R, DIR>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * NT;
        if ((b + 1) * NT <= nb || j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) st2(buf + widx[b] + r * NS, v[b][r]);
        }
    }
    __syncthreads();
}

template <int DIR, int NT, int N, int NS, int R, int... Rest, typename BT>
__device__ __forceinline__ void fft_passes_l(BT *buf, const double2 *twl, int tid) {
    stockham_stage_l<R, DIR, NT, N, NS>(buf, twl, tid);
    if constexpr (sizeof...(Rest) > 0) fft_passes_l<DIR, NT, N, NS * R, Rest...>(buf, twl + (NS > 1 ? NS : 0), tid);
}

// Number of LDS base twiddles of the passes from span NS on.
template <int NS, int... Rs>
struct TwCount {
    static constexpr int value = 0;
};
template <int NS, int R, int... Rest>
struct TwCount<NS, R, Rest...> {
    static constexpr int value = (NS > 1 ? NS : 0) + TwCount<NS * R, Rest...>::value;
};

// Copy the base rows out of the pass-major global table (entry (NS - 1) + k is w^k).
template <int NT, int NS, int R, int... Rest>
__device__ __forceinline__ void tw_base_load(double2 *twl, const double2 *__restrict__ tw, int tid) {
    if constexpr (NS > 1)
        for (int k = tid; k < NS; k += NT) twl[k] = tw[(NS - 1) + k];
    if constexpr (sizeof...(Rest) > 0) tw_base_load<NT, NS * R, Rest...>(twl + (NS > 1 ? NS : 0), tw, tid);
}

// Length of a compile-time transform, 0 for the runtime-planned one.
template <typename S>
struct FftLen {
    static constexpr int value = 0;
};
template <int N, int... Rs>
struct FftLen<FftSpec<N, Rs...>> {
    static constexpr int value = N;
};

template <int DIR, int NT, int PT, typename S>
struct FftRun;

template <int DIR, int NT, int PT>
struct FftRun<DIR, NT, PT, FftGeneric> {
    static constexpr int ntw = 0;  // twiddles stay in global memory
    __device__ __forceinline__ static void run(double2 *buf, const FftPlan &P, const double2 *__restrict__ tw, int tid, int nth) {
        fft_lds<DIR, NT, PT>(buf, P, tw, tid, nth);
    }
};

template <int DIR, int NT, int PT, int N, int... Rs>
struct FftRun<DIR, NT, PT, FftSpec<N, Rs...>> {
    static_assert(N <= NT * PT, "size class too small for the transform");
    static constexpr int ntw = TwCount<1, Rs...>::value;  // LDS base twiddles (run_l)
    __device__ __forceinline__ static void run(double2 *buf, const FftPlan &, const double2 *__restrict__ tw, int tid, int) {
        fft_passes_c<DIR, NT, N, 1, Rs...>(buf, tw, tid);
    }
    __device__ __forceinline__ static void load_tw(double2 *twl, const double2 *__restrict__ tw, int tid) {
        tw_base_load<NT, 1, Rs...>(twl, tw, tid);
    }
    // twl: the bases written by load_tw (visible to all threads); buf complex128 or complex64
    template <typename BT>
    __device__ __forceinline__ static void run_l(BT *buf, const double2 *twl, int tid) {
        fft_passes_l<DIR, NT, N, 1, Rs...>(buf, twl, tid);
    }
};
