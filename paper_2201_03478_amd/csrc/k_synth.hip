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
//   d^{l+1} = (alpha_l cos(theta) - beta_l) d^l - gamma_l d^{l-1}
//           = ((alpha_l - beta_l) - alpha_l y) d^l - gamma_l d^{l-1},  y = 1 - cos(theta)
// (the second form is evaluated, with y = 2 sin^2(theta/2) at full relative precision),
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
// The kernel runs the recursion on u^l = d^l / S_l with S_{l0} = S_{l0+1} = 1 and
// S_{l+1} = gamma_l S_{l-1}, which turns it into
//   u^{l+1} = (a_l cos(theta) - b_l) u^l - u^{l-1},  a_l = alpha_l S_l / S_{l+1},
//   b_l = beta_l S_l / S_{l+1},
// and folds S_l into the contraction weights: per d value one FMA forms
// (a_l - b_l) - a_l y, one FMA advances u and four FMAs contract it (both signs
// of m, real and imaginary parts).  S_l is O(1) (gamma_l -> 1; the alternating
// products of gamma telescope to about sqrt(l0 / l)), so u stays as well
// conditioned as d.  Every ring accumulates its scaled u unconditionally: while
// e < 0 the sums are meaningless, so they are cleared at the check where e
// reaches 0 (what the ring added before that is below 2^-248 in true units,
// i.e. nothing), and a ring that ends with e < 0 writes zero.  The check runs
// every 32 steps while some ring of the wave has e < 0; once all have e = 0
// (|d| <= 1, |u| = O(1) from then on) the loop runs without it.  Both loops
// cost the same six FMAs per d value.
//
// Every recursion runs on a northern ring (theta_j <= pi/2), where y is small
// next to the pole and exact in relative terms; the southern rings come from the
// reflection d^l_mk(pi - theta) = (-1)^{l+k} d^l_{-m,k}(theta).  So for m > 0 the
// column (m, k) runs two recursions per northern ring j:
//   R+ (the column (m, k)):  F_k(theta_j, m) and, mirrored, F_k(pi - theta_j, -m);
//   R- (the column (-m, k)): F_k(theta_j, -m) = sum_l (-1)^m conj(a_lm) conj(b_lk) d^l_{-m,k}
//                           and F_k(pi - theta_j, m) = sum_l (-1)^{l+k} a_lm conj(b_lk) d^l_{-m,k}.
// R- has beta_l of the opposite sign (alpha_l + beta_l in place of alpha_l - beta_l),
// the same gamma_l (so the same S_l) and the start value with the exponents of
// c and s exchanged and no sign.  For m = 0 the two coincide and R+ alone, with
// its mirror, covers every ring.  Rings past the equator are never recursed, so
// the rounding of cos(theta) next to the south pole cannot move the angle.
//
// R- runs on v^l = (-1)^l u^l_{-m,k}, for which
//   v^{l+1} = (a_l y - bn_l) v^l - v^{l-1},  bn_l = (alpha_l + beta_l) S_l / S_{l+1},
// and its two weights are those of R+ up to the sign (-1)^{l+k} and an exchange:
// (-1)^m conj(a) conj(b) = (-1)^{l+k} wm and (-1)^{l+k} a conj(b) = (-1)^{l+k} wp.
// So every lane forms q = fma(a_l, y', b'_l) with y' = -y, b' = b_l (R+) or
// y' = y, b' = -bn_l (R-), and accumulates wp v and wm v with the same weights;
// R- lanes read their sums in exchanged order, times (-1)^k.
//
// Layout: one 64-lane wave per (m, k, ring group); lanes 0-31 run R+ and lanes
// 32-63 run R- on the same northern rings, RPT rings per lane.  Recursion
// coefficients and weights for 64 consecutive l are built cooperatively in LDS
// (one l per lane, the square roots of alpha_l and gamma_l from a per-plan table of
// sqrt((l+1)^2 - x^2); S_l by a product scan over the lanes of each parity); a
// step reads a_l, wp and wm as broadcasts and b' from the lane's half.
#include "wigner_rec.h"

namespace {

using namespace wrec;

// Coefficients and weights of one step (l -> l+1), read from LDS: a = a_l, b = b'
// of the lane's recursion (R+ or R-, tp = 0 or 1), wp and wm.
struct RecCoef {
    double a, b;
    double2 wp, wm;
};

__device__ __forceinline__ RecCoef rec_load(int t, const double *cA, const double *cBt, const double2 *cWp,
                                            const double2 *cWm) {
    // cBt points at the lane's half of cB ([tp][64])
    return RecCoef{cA[t], cBt[t], cWp[t], cWm[t]};
}

// One recursion step for every ring of the lane: contract u^l (true value
// u S_l 2^{1200 e}, S_l folded into the weights) and advance to u^{l+1}.
template <int RPT>
__device__ __forceinline__ void rec_step(const RecCoef &c, const double *x, double *u, double *up, double2 *fp,
                                         double2 *fm) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        fp[r].x = fma(c.wp.x, u[r], fp[r].x);
        fp[r].y = fma(c.wp.y, u[r], fp[r].y);
        fm[r].x = fma(c.wm.x, u[r], fm[r].x);
        fm[r].y = fma(c.wm.y, u[r], fm[r].y);
        const double un = fma(fma(c.a, x[r], c.b), u[r], -up[r]);  // x holds y' = -+(1 - cos(theta))
        up[r] = u[r];
        u[r] = un;
    }
}

// Steps t0 .. t1-1.  Four steps per iteration with two coefficient sets in
// turn: the LDS reads of the next two steps are issued before the current two
// steps' arithmetic (a scheduling barrier keeps them there), and an even step
// count per iteration returns u / u_prev to the same registers, so neither the
// loads nor the recursion need register moves.
template <int RPT>
__device__ __forceinline__ void rec_steps(int t0, int t1, const double *cA, const double *cBt, const double2 *cWp,
                                          const double2 *cWm, const double *x, double *u, double *up, double2 *fp,
                                          double2 *fm) {
    const int te = t0 + ((t1 - t0) & ~3);
    if (te > t0) {
        RecCoef a0 = rec_load(t0, cA, cBt, cWp, cWm), a1 = rec_load(t0 + 1, cA, cBt, cWp, cWm);
        for (int t = t0; t < te; t += 4) {
            const RecCoef b0 = rec_load(t + 2, cA, cBt, cWp, cWm), b1 = rec_load(t + 3, cA, cBt, cWp, cWm);
            __builtin_amdgcn_sched_barrier(0);
            rec_step<RPT>(a0, x, u, up, fp, fm);
            rec_step<RPT>(a1, x, u, up, fp, fm);
            const int tn = t + 4 < te ? t + 4 : t;  // last iteration: harmless re-read
            a0 = rec_load(tn, cA, cBt, cWp, cWm);
            a1 = rec_load(tn + 1, cA, cBt, cWp, cWm);
            __builtin_amdgcn_sched_barrier(0);
            rec_step<RPT>(b0, x, u, up, fp, fm);
            rec_step<RPT>(b1, x, u, up, fp, fm);
        }
    }
    for (int t = te; t < t1; ++t) rec_step<RPT>(rec_load(t, cA, cBt, cWp, cWm), x, u, up, fp, fm);
}

// Up to 3 rings per lane the kernel fits 168 registers: three waves per SIMD.
template <int RPT, typename FT, bool TAB>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RPT <= 3 ? 3 : 2)))
k_ring_sums(const double2 *__restrict__ alm, const double2 *__restrict__ blm, FT *__restrict__ F,
            const double *__restrict__ sbin_m, const int *__restrict__ sbin_e,
            const double *__restrict__ rtab, const double2 *__restrict__ rroot, const double4 *__restrict__ ctab,
            const long long *__restrict__ ctab_off, int lmax, int kmax, int nring, int ngroups, int alm_lmax) {
    __shared__ double cA[64], cB[2 * 64];
    __shared__ double2 cWp[64], cWm[64];

    int b, g;  // b = column m (kmax + 1) + k
    xcd_column_group(blockIdx.x, (lmax + 1) * (kmax + 1), ngroups, b, g);
    const int k = b % (kmax + 1);
    const int m = b / (kmax + 1);
    const int lane = threadIdx.x;
    const int tp = lane >> 5, sub = lane & 31;  // recursion R+ (0) or R- (1); northern ring slot
    const int l0 = m > k ? m : k;
    const int mn = m < k ? m : k;
    const int nm = 2 * lmax + 1;
    const int nh = (nring + 1) / 2;  // northern rings, theta_j <= pi/2

    double x[RPT], u[RPT], up[RPT];
    int e[RPT];
    double2 fp[RPT], fm[RPT];

    const XN pref = {sbin_m[l0 * (kmax + 1) + mn], sbin_e[l0 * (kmax + 1) + mn]};
    const double pfe = (double)pref.e, pfm = log2(pref.m);  // log2 of the start prefactor
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 32 + sub;
        // R- has no work for m = 0 (R+ mirrors onto every ring) or on the equator ring of
        // an odd ring count (R+ writes both of its values)
        const bool on = j < nh && (tp == 0 || (m > 0 && j != nring - 1 - j));
        fp[r] = make_double2(0.0, 0.0);
        fm[r] = make_double2(0.0, 0.0);
        up[r] = 0.0;
        if (on) {
            start_value(rtab + 5 * j, m, k, pfe, pfm, x[r], u[r], e[r], tp == 1);
            if (tp == 0)
                x[r] = -x[r];  // y' = -y
            else if (l0 & 1)
                u[r] = -u[r];  // v^{l0} = (-1)^{l0} u^{l0}_{-m,k}
        } else {
            x[r] = 0.0;
            u[r] = 0.0;
            e[r] = 0;
        }
        scaled |= e[r] != 0;
    }
    bool fast = !__any(scaled);

    const size_t aoff = (size_t)m * (2 * alm_lmax + 1 - m) / 2;  // sky layout may have a larger lmax
    const size_t boff = (size_t)k * (2 * lmax + 1 - k) / 2;
    double s_prev = 1.0, s_cur = 1.0;  // S_{lc-1}, S_{lc} (S_{l0-1} := 1 only seeds the scan)
    // with the table, each chunk's entry is loaded during the previous chunk's steps
    const double4 *ccol = TAB ? ctab + ctab_off[m * (kmax + 1) + k] : nullptr;
    ChunkCoef cnext{0.0, 0.0, 0.0, 0.0};
    if (TAB) cnext = chunk_coefs_tab(ccol, l0, lane, l0, lmax);
    for (int lc = l0; lc <= lmax; lc += 64) {
        const ChunkCoef cc = TAB ? cnext : chunk_coefs(lc, lane, l0, lmax, m, k, rroot, s_prev, s_cur);
        __syncthreads();  // previous chunk's coefficients are consumed
        cA[lane] = cc.a;
        cB[lane] = cc.b;
        cB[64 + lane] = -cc.bn;
        chunk_weights(lc + lane, lmax, m, k, alm, blm, aoff, boff, cc.sl, [&](int which, double2 v) {
            if (which == 0) cWp[lane] = v;
            if (which == 1) cWm[lane] = v;  // the R- weights are these, exchanged and signed
        });
        __syncthreads();
        if (TAB) cnext = chunk_coefs_tab(ccol, lc + 64, lane, l0, lmax);  // in flight during the steps
        const int nl = (lmax - lc + 1) < 64 ? (lmax - lc + 1) : 64;
        const double *cBt = cB + 64 * tp;
        if (fast) {
            rec_steps<RPT>(0, nl, cA, cBt, cWp, cWm, x, u, up, fp, fm);
            continue;
        }
        // Rescaling is checked once per 32 steps: one step grows |u| by at most
        // ~2^11, so 32 steps stay inside the 2^424 left below overflow, and what a
        // ring accumulates between passing 2^600 and its rescale (true values below
        // 2^{-600 + 352}) is dropped harmlessly with the scaled sums.
        for (int t0 = 0; t0 < nl; t0 += 32) {
            const int t1 = t0 + 32 < nl ? t0 + 32 : nl;
            rec_steps<RPT>(t0, t1, cA, cBt, cWp, cWm, x, u, up, fp, fm);
            if (fast) continue;
            bool low = false;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (fabs(u[r]) > REC_BIG) {
                    u[r] = rec_down(u[r]);
                    up[r] = rec_down(up[r]);
                    e[r] += 1;
                    if (e[r] == 0) {  // in range from here on: drop the sums of the scaled values
                        fp[r] = make_double2(0.0, 0.0);
                        fm[r] = make_double2(0.0, 0.0);
                    }
                }
                low |= e[r] != 0;
            }
            fast = !__any(low);
        }
    }

#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 32 + sub;
        const int js = nring - 1 - j;  // the reflected (southern) ring
        if (e[r] != 0) {  // never in range: the true sums are below 2^-600
            fp[r] = make_double2(0.0, 0.0);
            fm[r] = make_double2(0.0, 0.0);
        }
        if (j < nh) {
            if (tp == 0) {  // F_k(theta_j, m); F_k(pi - theta_j, -m) (for m = 0: -m = m, skip the equator)
                st2(&F[((size_t)k * nm + (m + lmax)) * nring + j], fp[r]);
                if (m > 0 || js != j) st2(&F[((size_t)k * nm + (lmax - m)) * nring + js], fm[r]);
            } else if (m > 0 && js != j) {  // F_k(theta_j, -m) = (-1)^k sum wm v; F_k(pi - theta_j, m) = (-1)^k sum wp v
                const double sk = (k & 1) ? -1.0 : 1.0;
                st2(&F[((size_t)k * nm + (lmax - m)) * nring + j], cscale(fm[r], sk));
                st2(&F[((size_t)k * nm + (m + lmax)) * nring + js], cscale(fp[r], sk));
            }
        }
    }
}

}  // namespace

template <typename FT, bool TAB>
static void launch_ring_sums(sc_plan *p, const double *alm, const double *blm, FT *F) {
    const int nblk = (p->lmax + 1) * (p->kmax + 1) * p->ngroups;
    auto kern = k_ring_sums<4, FT, TAB>;
    switch (p->rpt) {
        case 1: kern = k_ring_sums<1, FT, TAB>; break;
        case 2: kern = k_ring_sums<2, FT, TAB>; break;
        case 3: kern = k_ring_sums<3, FT, TAB>; break;
        default: break;
    }
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(64), 0, p->stream, (const double2 *)alm, (const double2 *)blm, F,
                       p->sbin_m, p->sbin_e, p->rtab, p->rroot, p->ctab, p->ctab_off, p->lmax, p->kmax, p->nring,
                       p->ngroups, p->alm_lmax);
}

hipError_t sc_launch_ring_sums(sc_plan *p, const double *alm, const double *blm) {
    if (p->mid32) {
        if (p->ctab)
            launch_ring_sums<float2, true>(p, alm, blm, (float2 *)p->F);
        else
            launch_ring_sums<float2, false>(p, alm, blm, (float2 *)p->F);
    } else {
        if (p->ctab)
            launch_ring_sums<double2, true>(p, alm, blm, p->F);
        else
            launch_ring_sums<double2, false>(p, alm, blm, p->F);
    }
    return hipGetLastError();
}

namespace {

// One wave per (m, k) column: the chunk coefficients of every step, in the ring
// kernels' chunking (l0, l0 + 64, ...), so the table holds exactly the values they
// would compute.
__global__ void __launch_bounds__(64) k_rec_table(const double2 *__restrict__ rroot, double4 *__restrict__ ctab,
                                                  const long long *__restrict__ ctab_off, int lmax, int kmax) {
    const int col = blockIdx.x;
    const int m = col / (kmax + 1), k = col - m * (kmax + 1);
    const int l0 = m > k ? m : k;
    const int lane = threadIdx.x;
    double4 *out = ctab + ctab_off[col];
    double s_prev = 1.0, s_cur = 1.0;
    for (int lc = l0; lc <= lmax; lc += 64) {
        const ChunkCoef cc = chunk_coefs(lc, lane, l0, lmax, m, k, rroot, s_prev, s_cur);
        if (lc + lane <= lmax) out[lc - l0 + lane] = make_double4(cc.a, cc.b, cc.bn, cc.sl);
    }
}

}  // namespace

hipError_t sc_launch_rec_table(sc_plan *p) {
    if (!p->ctab) return hipSuccess;
    hipLaunchKernelGGL(k_rec_table, dim3((p->lmax + 1) * (p->kmax + 1)), dim3(64), 0, p->stream, p->rroot, p->ctab,
                       p->ctab_off, p->lmax, p->kmax);
    return hipGetLastError();
}

// Rings per lane: the fewest wasted lane slots with at most 4 rings per lane
// (more rings per lane spill registers).  A wave covers 32 RPT northern rings with
// each of the two recursions.
int sc_ring_groups(int nring, int rpt) {
    const int nh = (nring + 1) / 2;
    return (nh + 32 * rpt - 1) / (32 * rpt);
}

//
// Measured cost per ring slot (lmax 512, kmax 100) falls with the rings per lane
// (more independent recursions per wave hide the FMA latency) up to 3, where the
// kernel still runs three waves per SIMD: relative costs 1.65, 1.14, 1.0, 0.97 for
// 1 .. 4.  The layout minimises slots x cost.
void sc_choose_ring_layout(int nring, int *rpt, int *ngroups) {
    static const double cost[5] = {0.0, 1.65, 1.14, 1.0, 0.97};
    int best_r = 3, best_g = sc_ring_groups(nring, 3);
    double best = 1e300;
    for (int r = 3; r >= 1; --r) {  // 3 first: ties keep the larger count
        const int g = sc_ring_groups(nring, r);
        const double c = (double)g * 64 * r * cost[r];
        if (c < best) {
            best = c;
            best_r = r;
            best_g = g;
        }
    }
    {
        const int g = sc_ring_groups(nring, 4);
        if ((double)g * 64 * 4 * cost[4] < best) {
            best_r = 4;
            best_g = g;
        }
    }
    *rpt = best_r;
    *ngroups = best_g;
}
