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
__device__ XN xn_pow(double x, int n) {
    XN r = {0.5, 1};
    XN b = xn_norm(x, 0);
    while (n) {
        if (n & 1) r = xn_mul(r, b);
        b = xn_mul(b, b);
        n >>= 1;
    }
    return r;
}

constexpr int REC_STEP = 1200;  // rescaling exponent step
constexpr double REC_BIG = 0x1p600;
// 2^-1200 is below the FP64 range, so rescaling divides by 2^1200 through the
// exponent (ldexp), never through a multiplication by a constant.
__device__ __forceinline__ double rec_down(double v) { return ldexp(v, -REC_STEP); }


// Start value d^{l0}_{mk}(theta_j), l0 = max(m, k), theta_j = (j + 1/2) pi / nring,
// as a scaled FP64 value d and exponent step e <= 0 (true value d 2^{1200 e}):
//   d^l_{l k} = (-1)^{l-k} sqrt(C(2l, l+k)) c^{l+k} s^{l-k}   (m >= k)
//   d^l_{m l} =            sqrt(C(2l, l+m)) c^{l+m} s^{l-m}   (m <  k)
// c = cos(theta/2), s = sin(theta/2); pref = sqrt(C(2 l0, l0 + min(m, k))).
__device__ __forceinline__ void start_value(int j, int nring, int m, int k, XN pref, double &x, double &d, int &e) {
    const int l0 = m > k ? m : k, mn = m < k ? m : k;
    const double sgn = (m >= k && ((m - k) & 1)) ? -1.0 : 1.0;
    const double t = ((double)j + 0.5) / (double)nring;  // theta / pi
    x = cospi(t);
    const double ch = cospi(0.5 * t), sh = sinpi(0.5 * t);
    XN v = xn_mul(xn_mul(xn_pow(ch, l0 + mn), xn_pow(sh, l0 - mn)), pref);
    const int E = v.e;
    const int es = (E + REC_STEP / 2 >= 0) ? 0 : -((-(E + REC_STEP / 2) + REC_STEP - 1) / REC_STEP);
    e = es;
    d = sgn * ldexp(v.m, E - REC_STEP * es);
}

// Recursion coefficients for the step l -> l+1:
//   d^{l+1} = (A cos(theta) - B) d^l - C d^{l-1}.
__device__ __forceinline__ void rec_coefs(int l, double mm, double kk, double mk, double &A, double &B, double &C) {
    if (l == 0) {
        A = 1.0;
        B = 0.0;
        C = 0.0;
        return;
    }
    const double L = l, L1 = l + 1.0;
    const double q = sqrt((L1 * L1 - mm) * (L1 * L1 - kk));
    A = (2.0 * L + 1.0) * L1 / q;
    B = A * mk / (L * L1);
    C = L1 / L * sqrt((L * L - mm) * (L * L - kk)) / q;
}

}  // namespace wrec
