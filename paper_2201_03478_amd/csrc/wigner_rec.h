// wigner_rec.h -- pieces of the Wigner-d l-recursion shared by the ring-sum
// kernel and its adjoint: extended-exponent start values and the rescaling
// constants (see k_synth.hip for the recursion and its conventions).
#pragma once

#include "sc_common.h"

namespace wrec {

struct XN {
    double m;  // mantissa in [0.5, 1) (or 0)
    int e;     // value = m * 2^e
};

__device__ __forceinline__ XN xn_norm(double v, int e) {
    int ee;
    double mm = frexp(v, &ee);
    return {mm, e + ee};
}
__device__ __forceinline__ XN xn_mul(XN a, XN b) { return xn_norm(a.m * b.m, a.e + b.e); }
constexpr int REC_STEP = 1200;  // rescaling exponent step
constexpr double REC_BIG = 0x1p600;
// 2^-1200 is below the FP64 range, so rescaling divides by 2^1200 through the
// exponent (ldexp), never through a multiplication by a constant.
__device__ __forceinline__ double rec_down(double v) { return ldexp(v, -REC_STEP); }


// Start value d^{l0}_{mk}(theta_j), l0 = max(m, k), theta_j = (j + 1/2) pi / nring,
// as a scaled FP64 value d and exponent step e <= 0 (true value d 2^{1200 e}):
//   d^l_{l k} = (-1)^{l-k} sqrt(C(2l, l+k)) c^{l+k} s^{l-k}   (m >= k)
//   d^l_{m l} =            sqrt(C(2l, l+m)) c^{l+m} s^{l-m}   (m <  k)
// c = cos(theta/2), s = sin(theta/2).  It is formed in the log domain:
//   log2 |d| = pe + pm + P log2 c + Q log2 s,   P = l0 + min(m, k), Q = l0 - min(m, k),
// with sqrt(C(2 l0, l0 + min(m, k))) = 2^pe 2^pm (pe an integer, pm = log2 of its
// mantissa), log2 c and log2 s given per ring as double-double pairs (rt[1..4]),
// every product and sum carried with its rounding error (|log2 d| reaches 10^4
// at lmax 1800), then one exp2 of the fractional part: relative error ~1e-15.
// rt[0] = y = 1 - cos(theta_j) (returned in y).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
// With neg, the start value of the column (-m, k) instead (m, k >= 0):
//   d^l_{-l,k} = sqrt(C(2l, l-k)) c^{l-k} s^{l+k}   (m >= k),
//   d^l_{-m,l} = sqrt(C(2l, l-m)) c^{l-m} s^{l+m}   (m <  k),
// the same binomial with the exponents of c and s exchanged and no sign.
__device__ __forceinline__ void start_value(const double *__restrict__ rt, int m, int k, double pe, double pm,
                                            double &y, double &d, int &e, bool neg = false) {
    const int l0 = m > k ? m : k, mn = m < k ? m : k;
    const double sgn = (!neg && m >= k && ((m - k) & 1)) ? -1.0 : 1.0;
    y = rt[0];
    const double P = (double)(neg ? l0 - mn : l0 + mn), Q = (double)(neg ? l0 + mn : l0 - mn);
    const double p1 = P * rt[1], q1 = Q * rt[3];
    const double p1e = fma(P, rt[1], -p1) + P * rt[2];
    const double q1e = fma(Q, rt[3], -q1) + Q * rt[4];
    double s, se, t, te;
    two_sum(p1, q1, s, se);
    two_sum(s, pe, t, te);
    const double fl = floor(t);
    const double f = (t - fl) + (((se + te) + (p1e + q1e)) + pm);  // t - fl is exact; |f| < 3
    int de;
    const double mant = frexp(exp2(f), &de);  // |d| = mant 2^E, mant in [0.5, 1)
    const int E = (int)fl + de;
    const int es = (E + REC_STEP / 2 >= 0) ? 0 : -((-(E + REC_STEP / 2) + REC_STEP - 1) / REC_STEP);
    e = es;
    d = sgn * ldexp(mant, E - REC_STEP * es);
}

// Recursion coefficients for the step l -> l+1:
//   d^{l+1} = (A cos(theta) - B) d^l - C d^{l-1} = ((A - B) - A y) d^l - C d^{l-1},
// y = 1 - cos(theta).  The second form is the one evaluated: y keeps its full relative
// precision next to the poles, where cos(theta) rounded to FP64 would move the
// effective angle by up to 1e-16 / theta and the values at l by ~l^2 1e-16.
// A - B = A (l(l+1) - m k) / (l(l+1)) with the integer difference exact in FP64.
__device__ __forceinline__ void rec_coefs(int l, double mm, double kk, double mk, double &A, double &AmB,
                                          double &C) {
    if (l == 0) {
        A = 1.0;
        AmB = 1.0;
        C = 0.0;
        return;
    }
    const double L = l, L1 = l + 1.0;
    const double q = sqrt((L1 * L1 - mm) * (L1 * L1 - kk));
    A = (2.0 * L + 1.0) * L1 / q;
    AmB = A * ((L * L1 - mk) / (L * L1));
    C = L1 / L * sqrt((L * L - mm) * (L * L - kk)) / q;
}

}  // namespace wrec
