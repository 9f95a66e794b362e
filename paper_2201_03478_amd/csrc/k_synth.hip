// k_synth.hip -- ring sums of the spin transforms (FP64).
//
// For each beam order k (0..kmax), sky order m (0..lmax) and ring theta_j the
// kernel evaluates
//     F_k(theta_j,  m)        = sum_l a_lm conj(b_lk) d^l_mk(theta_j)
//     F_k(pi - theta_j, -m)   = sum_l (-1)^{l+k+m} conj(a_lm) conj(b_lk) d^l_mk(theta_j)
// i.e. the inner sum of Eq. 7 / Eq. 9 of Galloway et al. (2022, Sec. 2.1) on
// a ring, before its azimuthal Fourier synthesis.  The second line follows from
// d^l_{-m,k}(pi - theta) = (-1)^{l+k} d^l_mk(theta) and a_{l,-m} = (-1)^m conj(a_lm)
// (real sky), so one recursion per (k, m >= 0) serves both signs of m; rings
// are placed symmetrically, theta_{nring-1-j} = pi - theta_j.
//
// d^l_mk(theta) comes from the three-term recursion in l,
//   d^{l+1} = (alpha_l cos(theta) - beta_l) d^l - gamma_l d^{l-1},
//   alpha_l = (2l+1)(l+1) / sqrt(((l+1)^2-m^2)((l+1)^2-k^2)),
//   beta_l  = alpha_l m k / (l(l+1)),
//   gamma_l = (l+1)/l sqrt((l^2-m^2)(l^2-k^2)) / sqrt(((l+1)^2-m^2)((l+1)^2-k^2)),
// started at l0 = max(m, k) from the closed forms
//   d^l_{l k} = (-1)^{l-k} sqrt(C(2l, l+k)) c^{l+k} s^{l-k}   (m >= k),
//   d^l_{m l} =            sqrt(C(2l, l+m)) c^{l+m} s^{l-m}   (m <  k),
// c = cos(theta/2), s = sin(theta/2).  Start values underflow FP64 near the
// poles (down to ~1e-1440 at l = 512), so they are formed as extended-exponent
// numbers and the recursion runs on a value scaled by 2^{-1200 e}: while
// e < 0 the true value is below 2^-600 and contributes nothing; whenever the
// scaled value passes 2^600 it is rescaled and e incremented.  Once e = 0 the
// true values are bounded by 1 and no further rescaling happens.
//
// Layout: one 64-lane wave per (m, k, ring group); each lane carries RPT
// rings.  Recursion coefficients and weights for 64 consecutive l are built
// cooperatively in LDS (one l per lane) and read as broadcasts.
#include "wigner_rec.h"

namespace {

using namespace wrec;

// One recursion step for every ring of the lane: contract d^l (its true value
// d * 2^{1200 e}; below 2^-600 while e < 0, i.e. nothing) and advance to d^{l+1}.
template <int RPT>
__device__ __forceinline__ void rec_step(int t, const double *cA, const double *cB, const double *cC,
                                         const double2 *cWp, const double2 *cWm, const double *x, double *d,
                                         double *dp, const int *e, double2 *fp, double2 *fm) {
    const double A = cA[t], B = cB[t], C = cC[t];
    const double2 wp = cWp[t], wm = cWm[t];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const double dd = ldexp(d[r], REC_STEP * e[r]);
        fp[r].x = fma(wp.x, dd, fp[r].x);
        fp[r].y = fma(wp.y, dd, fp[r].y);
        fm[r].x = fma(wm.x, dd, fm[r].x);
        fm[r].y = fma(wm.y, dd, fm[r].y);
        const double dn = fma(fma(A, x[r], -B), d[r], -C * dp[r]);
        dp[r] = d[r];
        d[r] = dn;
    }
}

template <int RPT>
__global__ void __launch_bounds__(64)
k_ring_sums(const double2 *__restrict__ alm, const double2 *__restrict__ blm, double2 *__restrict__ F,
            const double *__restrict__ sbin_m, const int *__restrict__ sbin_e, int lmax, int kmax, int nring,
            int ngroups, int alm_lmax) {
    __shared__ double cA[64], cB[64], cC[64];
    __shared__ double2 cWp[64], cWm[64];

    int b = blockIdx.x;
    const int g = b % ngroups;
    b /= ngroups;
    const int k = b % (kmax + 1);
    const int m = b / (kmax + 1);
    const int lane = threadIdx.x;
    const int l0 = m > k ? m : k;
    const int mn = m < k ? m : k;
    const int nm = 2 * lmax + 1;

    double x[RPT], d[RPT], dp[RPT];
    int e[RPT];
    double2 fp[RPT], fm[RPT];

    const XN pref = {sbin_m[l0 * (kmax + 1) + mn], sbin_e[l0 * (kmax + 1) + mn]};
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 64 + lane;
        fp[r] = make_double2(0.0, 0.0);
        fm[r] = make_double2(0.0, 0.0);
        dp[r] = 0.0;
        if (j < nring) {
            start_value(j, nring, m, k, pref, x[r], d[r], e[r]);
        } else {
            x[r] = 0.0;
            d[r] = 0.0;
            e[r] = 0;
        }
    }

    const double mm = (double)m * m, kk = (double)k * k, mk = (double)m * k;
    const size_t aoff = (size_t)m * (2 * alm_lmax + 1 - m) / 2;  // sky layout may have a larger lmax
    const size_t boff = (size_t)k * (2 * lmax + 1 - k) / 2;
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
            const double2 wm = cscale(cmul(cconj(a), cconj(bb)), s);
            cA[lane] = A;
            cB[lane] = B;
            cC[lane] = C;
            cWp[lane] = wp;
            cWm[lane] = wm;
        }
        __syncthreads();
        const int nl = (lmax - lc + 1) < 64 ? (lmax - lc + 1) : 64;
        // Rescaling is checked once per 8 steps: one step grows |d| by at most
        // ~2^10 (alpha_l <= l0 + 1), far inside the 2^424 left below overflow.
        for (int t0 = 0; t0 < nl; t0 += 8) {
            const int t1 = t0 + 8 < nl ? t0 + 8 : nl;
#pragma unroll 2
            for (int t = t0; t < t1; ++t) rec_step<RPT>(t, cA, cB, cC, cWp, cWm, x, d, dp, e, fp, fm);
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (fabs(d[r]) > REC_BIG) {
                    d[r] *= REC_DOWN;
                    dp[r] *= REC_DOWN;
                    e[r] += 1;
                }
            }
        }
    }

#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 64 + lane;
        if (j < nring) {
            F[((size_t)k * nm + (m + lmax)) * nring + j] = fp[r];
            if (m > 0) F[((size_t)k * nm + (lmax - m)) * nring + (nring - 1 - j)] = fm[r];
        }
    }
}

}  // namespace

#define SC_RING_CASE(R)                                                                                      \
    case R:                                                                                                  \
        hipLaunchKernelGGL(k_ring_sums<R>, dim3(nblk), dim3(64), 0, p->stream, (const double2 *)alm,         \
                           (const double2 *)blm, p->F, p->sbin_m, p->sbin_e, p->lmax, p->kmax, p->nring,      \
                           p->ngroups, p->alm_lmax);                                                         \
        break;

hipError_t sc_launch_ring_sums(sc_plan *p, const double *alm, const double *blm) {
    const int nblk = (p->lmax + 1) * (p->kmax + 1) * p->ngroups;
    switch (p->rpt) {
        SC_RING_CASE(1)
        SC_RING_CASE(2)
        SC_RING_CASE(3)
        default:
        SC_RING_CASE(4)
    }
    return hipGetLastError();
}

// Rings per lane: the fewest wasted lane slots with at most 4 rings per lane
// (more rings per lane spill registers).
void sc_choose_ring_layout(int nring, int *rpt, int *ngroups) {
    int best_r = 1, best_g = (nring + 63) / 64, best_w = 1 << 30;
    for (int r = 4; r >= 1; --r) {
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
