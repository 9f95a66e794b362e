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

// Step l = lc + lane of a chunk of 64 steps of the normalised recursions on
// u^l = d^l / S_l (S_{l0} = S_{l0+1} = 1, S_{l+1} = gamma_l S_{l-1}):
//   u^{l+1} = (b - a y) u^l - u^{l-1},  a = alpha_l S_l / S_{l+1},
// b = (alpha_l - beta_l) S_l / S_{l+1} for the column (m, k) (R+) and
// bn = (alpha_l + beta_l) S_l / S_{l+1} for the column (-m, k) (R-).  alpha, beta
// and gamma come from the plan's root table sqrt((l+1)^2 - x^2) and its
// reciprocal; S_l from a product scan over the lanes of each parity, carried
// across chunks in s_prev = S_{lc-1}, s_cur = S_{lc}.  Called by all 64 lanes.
struct ChunkCoef {
    double a, b, bn, sl;  // sl = S_l, the factor of the contraction weights
};

__device__ __forceinline__ ChunkCoef chunk_coefs(int lc, int lane, int l0, int lmax, int m, int k,
                                                 const double2 *__restrict__ rroot, double &s_prev, double &s_cur) {
    const int l = lc + lane;
    const double mk = (double)m * k;
    double A = 1.0, B = 0.0, Bn = 0.0, C = 1.0;
    if (l <= lmax) {
        if (l == 0) {
            B = 1.0;
            Bn = 1.0;
            C = 0.0;
        } else {
            // q = r(m, l) r(k, l) with r(x, l) = sqrt((l+1)^2 - x^2), and
            // sqrt((l^2-m^2)(l^2-k^2)) = r(m, l-1) r(k, l-1)
            const double2 tm = rroot[(size_t)m * (lmax + 1) + l], tk = rroot[(size_t)k * (lmax + 1) + l];
            const double2 pm = rroot[(size_t)m * (lmax + 1) + l - 1], pk = rroot[(size_t)k * (lmax + 1) + l - 1];
            const double L = (double)l, L1 = L + 1.0;
            const double rq = tm.y * tk.y;
            const double inv = 1.0 / (L * L1);
            A = (2.0 * L + 1.0) * L1 * rq;
            B = A * ((L * L1 - mk) * inv);   // alpha - beta, the integer difference exact
            Bn = A * ((L * L1 + mk) * inv);  // alpha + beta
            C = L1 * L1 * inv * (pm.x * pk.x) * rq;
        }
    }
    if (l == l0) C = 1.0;  // S_{l0+1} := 1 (gamma_{l0} = 0)
    // T = S_{l+1} = gamma_l S_{l-1}: inclusive product over the lanes of this
    // lane's parity, times the carried S_{lc-1} (even lanes) or S_{lc} (odd).
    double T = C;
#pragma unroll
    for (int off = 2; off < 64; off <<= 1) {
        const double v = __shfl_up(T, off);
        if (lane >= off) T *= v;
    }
    T *= (lane & 1) ? s_cur : s_prev;
    double Sl = __shfl_up(T, 1);  // S_l
    if (lane == 0) Sl = s_cur;
    s_prev = __shfl(T, 62);  // S_{lc+63} and S_{lc+64} for the next chunk
    s_cur = __shfl(T, 63);
    const double ratio = Sl / T;
    return ChunkCoef{A * ratio, B * ratio, Bn * ratio, Sl};
}

// The chunk coefficients depend on (m, k, l) only, so a plan can hold them for every
// column (k_rec_table, entry l - l0 of column (m, k) = (a, b, bn, S_l) as chunk_coefs
// returns them, with the same chunking from l0): one coalesced load per lane instead
// of the root-table loads, two divisions and the product scan, in every wave of every
// synthesis.  Zero past lmax (no step reads those; the weights there are zero).
__device__ __forceinline__ ChunkCoef chunk_coefs_tab(const double4 *__restrict__ col, int lc, int lane, int l0,
                                                     int lmax) {
    const int l = lc + lane;
    if (l > lmax) return ChunkCoef{0.0, 0.0, 0.0, 0.0};
    const double4 q = col[l - l0];
    return ChunkCoef{q.x, q.y, q.z, q.w};
}

// Contraction weights of step l (zero past lmax), each times S_l:
//   R+: wp = a_lm conj(b_lk)                    -> F_k(theta_j, m)
//       wm = (-1)^{l+k+m} conj(a_lm) conj(b_lk) -> F_k(pi - theta_j, -m)
//   R-: wpn = (-1)^m conj(a_lm) conj(b_lk)      -> F_k(theta_j, -m)
//       wmn = (-1)^{l+k} a_lm conj(b_lk)        -> F_k(pi - theta_j, m)
// (Im a_l0 and Im b_l0 are ignored.)  `put(which, value)` receives them in that order.
template <typename Put>
__device__ __forceinline__ void chunk_weights(int l, int lmax, int m, int k, const double2 *__restrict__ alm,
                                              const double2 *__restrict__ blm, size_t aoff, size_t boff, double sl,
                                              Put put) {
    double2 a = make_double2(0.0, 0.0), bb = a;
    if (l <= lmax) {
        a = alm[aoff + l];
        bb = blm[boff + l];
        if (m == 0) a.y = 0.0;
        if (k == 0) bb.y = 0.0;
    }
    const double2 wp = cscale(cmul(a, cconj(bb)), sl);
    put(0, wp);
    const double2 cacb = cscale(cmul(cconj(a), cconj(bb)), sl);
    put(1, cscale(cacb, ((l + k + m) & 1) ? -1.0 : 1.0));
    put(2, cscale(cacb, (m & 1) ? -1.0 : 1.0));
    put(3, cscale(wp, ((l + k) & 1) ? -1.0 : 1.0));
}

}  // namespace wrec
