// k_synth_mixed.hip -- ring sums in mixed precision (the precision variant).
//
// Same quantity as k_synth.hip (the inner sums of Eqs. 7/9, Galloway et al.
// 2022, Sec. 2.1, on both signs of m):
//     F_k(theta_j, m)       = sum_l a_lm conj(b_lk) d^l_mk(theta_j)
//     F_k(pi - theta_j, -m) = sum_l (-1)^{l+k+m} conj(a_lm) conj(b_lk) d^l_mk(theta_j)
// with the arithmetic split as:
//  * start values d^{l0}_mk in FP64 extended-exponent form (as in the FP64
//    kernel), then rounded to an FP32 value with a 2^{128 e} exponent step;
//  * the three-term l-recursion in FP32 on the VALU, written as
//      d^{l+1} = ((alpha - beta) - alpha y) d^l - gamma d^{l-1},  y = 1 - cos(theta)
//    with alpha - beta formed in FP64 and y = 2 sin^2(theta/2): near the poles
//    cos(theta) rounded to FP32 would keep only a few digits of 1 - cos(theta),
//    which (alpha cos(theta) - beta) then cancels.  Coefficients are rounded to
//    FP32; the value is rescaled by 2^-128 whenever |d| passes 2^64 (checked
//    every 4 steps; one step grows |d| by at most ~2^11);
//  * the contraction on the matrix cores: v_mfma_f32_4x4x1_16b_f32 computes
//    16 independent 4x4 outer products.  Lane 4b + i supplies d of its own ring
//    (A of block b, row i), lane 4b + j supplies weight component j of the
//    current l (B, column j: Re w+, Im w+, Re w-, Im w-), and the accumulator
//    of lane 4b + j, register i, collects component j for ring 4b + i.  FP32
//    products, FP32 accumulation, no operand reshuffling; the VALU only runs
//    the recursion.
// The FP32 recursion's error grows with l (relative ~1e-6 at l ~ 1000); the
// result is reported against the FP64 oracle.
#include "wigner_rec.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

using namespace wrec;

constexpr int MX_STEP = 128;          // FP32 rescaling exponent step
constexpr float MX_BIG = 0x1p64f;  // rescaling divides by 2^128 through the exponent (ldexpf)

template <int RPT>
__global__ void __launch_bounds__(64)
k_ring_sums_mixed(const double2 *__restrict__ alm, const double2 *__restrict__ blm, double2 *__restrict__ F,
                  const double *__restrict__ sbin_m, const int *__restrict__ sbin_e,
            const double *__restrict__ rtab, int lmax, int kmax, int nring,
                  int ngroups, int alm_lmax) {
    __shared__ float cA[64], cB[64], cC[64];
    __shared__ float cW[64][4];
    __shared__ float Fs[RPT][64][4];

    int b = blockIdx.x;
    const int g = b % ngroups;
    b /= ngroups;
    const int k = b % (kmax + 1);
    const int m = b / (kmax + 1);
    const int lane = threadIdx.x;
    const int l0 = m > k ? m : k;
    const int mn = m < k ? m : k;
    const int nm = 2 * lmax + 1;

    float x[RPT], d[RPT], dp[RPT];  // x holds y = 1 - cos(theta)
    int e[RPT];
    floatx4 acc[RPT];
    const XN pref = {sbin_m[l0 * (kmax + 1) + mn], sbin_e[l0 * (kmax + 1) + mn]};
    const double pfe = (double)pref.e, pfm = log2(pref.m);  // log2 of the start prefactor
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 64 + lane;
        acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        dp[r] = 0.f;
        x[r] = 0.f;
        d[r] = 0.f;
        e[r] = 0;
        if (j < nring) {
            double xd, dd;
            int ed;
            start_value(rtab + 5 * j, m, k, pfe, pfm, xd, dd, ed);
            // true value dd 2^{1200 ed}: re-express as an FP32 value with a 2^{128 e} step
            int E;
            const double mant = frexp(dd, &E);
            const long long Et = (long long)E + (long long)REC_STEP * ed;
            const long long es = (Et + MX_STEP / 2 >= 0) ? 0 : -((-(Et + MX_STEP / 2) + MX_STEP - 1) / MX_STEP);
            if (es < -1000) {
                e[r] = -1000;  // far below anything that reaches l = lmax
            } else {
                e[r] = (int)es;
                d[r] = (float)ldexp(mant, (int)(Et - (long long)MX_STEP * es));
            }
            const double sh = sinpi(0.5 * ((double)j + 0.5) / (double)nring);
            x[r] = (float)(2.0 * sh * sh);  // y = 1 - cos(theta), full relative precision
            (void)xd;
        }
    }

    const double mm = (double)m * m, kk = (double)k * k, mk = (double)m * k;
    const size_t aoff = (size_t)m * (2 * alm_lmax + 1 - m) / 2;  // sky layout may have a larger lmax
    const size_t boff = (size_t)k * (2 * lmax + 1 - k) / 2;
    const int comp = lane & 3;
    for (int lc = l0; lc <= lmax; lc += 64) {
        const int l = lc + lane;
        __syncthreads();
        if (l <= lmax) {
            double A, B, C;
            rec_coefs(l, mm, kk, mk, A, B, C);
            double2 a = alm[aoff + l];
            double2 bb = blm[boff + l];
            if (m == 0) a.y = 0.0;
            if (k == 0) bb.y = 0.0;
            const double2 wp = cmul(a, cconj(bb));
            const double s = ((l + k + m) & 1) ? -1.0 : 1.0;
            const double2 wm = m > 0 ? cscale(cmul(cconj(a), cconj(bb)), s) : make_double2(0.0, 0.0);
            cA[lane] = (float)A;
            cB[lane] = (float)B;  // alpha - beta, formed in FP64 by rec_coefs
            cC[lane] = (float)C;
            cW[lane][0] = (float)wp.x;
            cW[lane][1] = (float)wp.y;
            cW[lane][2] = (float)wm.x;
            cW[lane][3] = (float)wm.y;
        }
        __syncthreads();
        const int nl = (lmax - lc + 1) < 64 ? (lmax - lc + 1) : 64;
        for (int t0 = 0; t0 < nl; t0 += 4) {
            const int t1 = t0 + 4 < nl ? t0 + 4 : nl;
            for (int t = t0; t < t1; ++t) {
                const float A = cA[t], B = cB[t], C = cC[t];
                const float w = cW[t][comp];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const float dd = ldexpf(d[r], MX_STEP * e[r]);
                    acc[r] = __builtin_amdgcn_mfma_f32_4x4x1f32(dd, w, acc[r], 0, 0, 0);
                    const float dn = fmaf(fmaf(-A, x[r], B), d[r], -C * dp[r]);
                    dp[r] = d[r];
                    d[r] = dn;
                }
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (fabsf(d[r]) > MX_BIG) {
                    d[r] = ldexpf(d[r], -MX_STEP);
                    dp[r] = ldexpf(dp[r], -MX_STEP);
                    e[r] += 1;
                }
            }
        }
    }

    // lane 4q + j holds component j of rings 4q + i in register i: regroup per ring
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) Fs[r][(lane & ~3) + i][comp] = acc[r][i];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 64 + lane;
        if (j < nring) {
            const float *f = Fs[r][lane];
            F[((size_t)k * nm + (m + lmax)) * nring + j] = make_double2((double)f[0], (double)f[1]);
            if (m > 0)
                F[((size_t)k * nm + (lmax - m)) * nring + (nring - 1 - j)] = make_double2((double)f[2], (double)f[3]);
        }
    }
}

}  // namespace

#define SC_MIXED_CASE(R)                                                                                     \
    case R:                                                                                                  \
        hipLaunchKernelGGL(k_ring_sums_mixed<R>, dim3(nblk), dim3(64), 0, p->stream, (const double2 *)alm,   \
                           (const double2 *)blm, p->F, p->sbin_m, p->sbin_e, p->rtab, p->lmax, p->kmax, p->nring,      \
                           p->ngroups_mx, p->alm_lmax);                                                     \
        break;

hipError_t sc_launch_ring_sums_mixed(sc_plan *p, const double *alm, const double *blm) {
    const int nblk = (p->lmax + 1) * (p->kmax + 1) * p->ngroups_mx;
    switch (p->rpt_mx) {
        SC_MIXED_CASE(1)
        SC_MIXED_CASE(2)
        SC_MIXED_CASE(3)
        SC_MIXED_CASE(4)
        SC_MIXED_CASE(5)
        SC_MIXED_CASE(6)
        SC_MIXED_CASE(7)
        default:
        SC_MIXED_CASE(8)
    }
    return hipGetLastError();
}

// Rings per lane for the FP32 kernel (half the registers of FP64: up to 8).
void sc_choose_ring_layout_mixed(int nring, int *rpt, int *ngroups) {
    int best_r = 1, best_g = (nring + 63) / 64, best_w = 1 << 30;
    for (int r = 8; r >= 1; --r) {
        const int g = (nring + 64 * r - 1) / (64 * r);
        const int waste = g * 64 * r - nring;
        if (waste < best_w) {
            best_w = waste;
            best_r = r;
            best_g = g;
        }
    }
    *rpt = best_r;
    *ngroups = best_g;
}
