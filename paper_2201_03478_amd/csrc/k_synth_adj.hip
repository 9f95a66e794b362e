// k_synth_adj.hip -- adjoint of the ring sums (gradient w.r.t. the sky a_lm).
//
// The forward ring sums are (k_synth.hip)
//     F_k(theta_j, m)      = sum_l a_lm conj(b_lk) d^l_mk(theta_j)
//     F_k(pi - theta_j, -m) = sum_l (-1)^{l+k+m} conj(a_lm) conj(b_lk) d^l_mk(theta_j),
// the inner sums of Eqs. 7/9 of Galloway et al. (2022, Sec. 2.1).  Given the
// ring-sum gradients F_adj (from the adjoint transforms), with the real inner
// product Re sum conj(u) v, the gradient g = dL/dRe a_lm + i dL/dIm a_lm is
//     Q+(l) = sum_j d^l_mk(theta_j) F_adj_k(theta_j, m),
//     Q-(l) = sum_j d^l_mk(theta_j) F_adj_k(pi - theta_j, -m),
//     g_lm  = sum_k [ Q+ b_lk + (-1)^{l+k+m} conj(Q- b_lk) ]      (m > 0),
//     g_l0  = sum_k Re(Q+ b_lk)                                  (m = 0).
// The d values come from the same recursions and start values as the forward
// kernel, on northern rings only: lanes 0-31 run the column (m, k) (R+) for the
// rings theta_j <= pi/2, lanes 32-63 the column (-m, k) (R-) on the same rings,
// which by d^l_mk(pi - theta) = (-1)^{l+k} d^l_{-m,k}(theta) gives the southern
// rings.  R- runs on (-1)^l d^l_{-m,k}, whose recursion has the coefficient
// -((alpha + beta) - alpha y) and the same gamma, so that its products with the
// ring-sum gradients (times (-1)^k, folded into them at load) add to the same
// per-l sums as R+'s:
//     Q+(l) = sum_{j north} [d^l_mk(theta_j) F_adj(theta_j, m) + (-1)^k dt F_adj(pi - theta_j, m)],
//     Q-(l) = sum_{j north} [d^l_mk(theta_j) F_adj(pi - theta_j, -m) + (-1)^k dt F_adj(theta_j, -m)],
// dt = (-1)^l d^l_{-m,k}(theta_j).  The sums over rings are reductions across lanes for every l: each
// lane adds its rings' products, writes the 4 real partials of each l to a
// padded LDS buffer, and every 8 l the buffer is reduced by reading it
// transposed (two lanes per (l, value) row).  One wave per ring group; the
// waves of a workgroup are the groups of one (k, m) and are combined in LDS.
// Per-k contributions go to GA[k][alm index]; a second kernel sums over k in a
// fixed order (deterministic).  Columns with more than 2048 rings are split into
// slabs of rings, one workgroup each, whose partial sums go to separate copies of
// GA and are added by the same fixed-order reduction (no atomics).
//
// The same Q+- give the gradient with respect to the beam (BEAM = true): the
// TOD is bilinear, and with the sky gradient above L = Re sum conj(g_lm) a_lm
// is, as a function of b,
//     L = Re sum_{l,k,m>0} [conj(b_lk) conj(Q+) a_lm + b_lk (-1)^{l+k+m} Q- a_lm]
//       + Re sum_{l,k} b_lk Q+(m = 0) a_l0,
// so h_lk = dL/dRe b_lk + i dL/dIm b_lk = sum_m [conj(Q+) a_lm +
// (-1)^{l+k+m} conj(Q- a_lm)] (the Q- term for m > 0), real for k = 0.  Per-m
// contributions go to GB[m][blm index] and are summed over m in a fixed order.
#include "wigner_rec.h"

namespace {

using namespace wrec;

constexpr int ADJ_FLUSH = 8;   // l steps per LDS flush
constexpr int ADJ_ROW = 65;    // padded row length (doubles) of the partial buffer

template <int RPT, bool BEAM>
__global__ void __launch_bounds__(1024)
k_ring_sums_adjoint(const double2 *__restrict__ FA, const double2 *__restrict__ coefs, double2 *__restrict__ GA,
                    const double *__restrict__ sbin_m, const int *__restrict__ sbin_e,
                    const double *__restrict__ rtab, int lmax, int kmax, int nring, int alm_lmax, int nslab,
                    int per) {
    // coefs: the beam b_lk (sky gradient into GA[k]) or, with BEAM, the sky a_lm
    // in the alm_lmax layout (beam gradient into GA[m], blm layout)
    extern __shared__ __attribute__((aligned(16))) double adj_smem[];
    const int nw = blockDim.x >> 6;
    double *cA = adj_smem, *cB = cA + 128, *cC = cB + 128;  // [64][2] per recursion, [64]
    double *Qw = cC + 64;                                    // [nw][64][4]
    double *PB = Qw + nw * 64 * 4;                                          // [nw][4][FLUSH][ROW]
    const int slab = blockIdx.x % nslab;  // rings [slab per, slab per + per)
    const int b = blockIdx.x / nslab;
    const int k = b % (kmax + 1);
    const int m = b / (kmax + 1);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tp = lane >> 5, sub = lane & 31;  // recursion R+ (0) or R- (1); northern ring slot
    const int nh = (nring + 1) / 2;
    const int l0 = m > k ? m : k;
    const int mn = m < k ? m : k;
    const int nm = 2 * lmax + 1;
    const size_t aoff = (size_t)m * (2 * lmax + 1 - m) / 2;
    const size_t nalm = (size_t)(lmax + 1) * (lmax + 2) / 2;
    const size_t boff = (size_t)k * (2 * lmax + 1 - k) / 2;
    const size_t nblm = (size_t)(kmax + 1) * (2 * lmax + 2 - kmax) / 2;
    // output column: (l, m) of GA[k] for the sky gradient, (l, k) of GA[m] for the beam
    double2 *gk = BEAM ? GA + ((size_t)slab * (lmax + 1) + m) * nblm + boff
                       : GA + ((size_t)slab * (kmax + 1) + k) * nalm + aoff;
    // orders below l0 have no d^l_mk: their contribution is zero
    for (int l = (BEAM ? k : m) + tid; l < l0 && l <= lmax; l += blockDim.x) gk[l] = make_double2(0.0, 0.0);
    if (l0 > lmax) return;

    double x[RPT], d[RPT], dp[RPT];
    int e[RPT];
    double2 fap[RPT], fam[RPT];
    const XN pref = {sbin_m[l0 * (kmax + 1) + mn], sbin_e[l0 * (kmax + 1) + mn]};
    const double pfe = (double)pref.e, pfm = log2(pref.m);  // log2 of the start prefactor
    const double sk = (k & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int jl = (w * RPT + r) * 32 + sub;  // northern ring within the slab
        const int j = slab * per + jl, js = nring - 1 - j;
        dp[r] = 0.0;
        fap[r] = make_double2(0.0, 0.0);
        fam[r] = make_double2(0.0, 0.0);
        if (jl < per && j < nh && (tp == 0 || js != j)) {  // R- skips the equator ring of an odd count
            start_value(rtab + 5 * j, m, k, pfe, pfm, x[r], d[r], e[r], tp == 1);
            if (tp == 0) {
                fap[r] = FA[((size_t)k * nm + (m + lmax)) * nring + j];
                if (m > 0) fam[r] = FA[((size_t)k * nm + (lmax - m)) * nring + js];
            } else {
                if (l0 & 1) d[r] = -d[r];  // (-1)^l d^l_{-m,k} at l = l0
                fap[r] = cscale(FA[((size_t)k * nm + (m + lmax)) * nring + js], sk);
                if (m > 0) fam[r] = cscale(FA[((size_t)k * nm + (lmax - m)) * nring + j], sk);
            }
        } else {
            x[r] = 0.0;
            d[r] = 0.0;
            e[r] = 0;
        }
    }

    double *pbw = PB + (size_t)w * 4 * ADJ_FLUSH * ADJ_ROW;
    const double mm = (double)m * m, kk = (double)k * k, mk = (double)m * k;
    for (int lc = l0; lc <= lmax; lc += 64) {
        __syncthreads();  // previous chunk's coefficients and Qw are consumed
        if (tid < 64 && lc + tid <= lmax) {
            double A, B, C, Bn, Cn;
            rec_coefs(lc + tid, mm, kk, mk, A, B, C);      // B = alpha - beta
            rec_coefs(lc + tid, mm, kk, -mk, A, Bn, Cn);   // Bn = alpha + beta (the column (-m, k))
            cA[2 * tid] = -A;  // R+: (alpha - beta) - alpha y
            cB[2 * tid] = B;
            cA[2 * tid + 1] = A;  // R- on (-1)^l d: -((alpha + beta) - alpha y)
            cB[2 * tid + 1] = -Bn;
            cC[tid] = C;
        }
        __syncthreads();
        const int nl = (lmax - lc + 1) < 64 ? (lmax - lc + 1) : 64;
        for (int t0 = 0; t0 < nl; t0 += ADJ_FLUSH) {
            const int t1 = t0 + ADJ_FLUSH < nl ? t0 + ADJ_FLUSH : nl;
            for (int t = t0; t < t1; ++t) {
                const double A = cA[2 * t + tp], B = cB[2 * t + tp], C = cC[t];
                double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const double dd = ldexp(d[r], REC_STEP * e[r]);
                    p0 = fma(dd, fap[r].x, p0);
                    p1 = fma(dd, fap[r].y, p1);
                    p2 = fma(dd, fam[r].x, p2);
                    p3 = fma(dd, fam[r].y, p3);
                    const double dn = fma(fma(A, x[r], B), d[r], -C * dp[r]);  // x: 1 - cos theta
                    dp[r] = d[r];
                    d[r] = dn;
                }
                double *row = pbw + (t - t0) * ADJ_ROW + lane;
                row[0 * ADJ_FLUSH * ADJ_ROW] = p0;
                row[1 * ADJ_FLUSH * ADJ_ROW] = p1;
                row[2 * ADJ_FLUSH * ADJ_ROW] = p2;
                row[3 * ADJ_FLUSH * ADJ_ROW] = p3;
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (fabs(d[r]) > REC_BIG) {
                    d[r] = rec_down(d[r]);
                    dp[r] = rec_down(dp[r]);
                    e[r] += 1;
                }
            }
            // wave-local transpose-reduce: row (v, tt) summed by lanes 2 row, 2 row + 1
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            const int rr = lane >> 1, half = lane & 1;  // rr in [0, 32): v = rr / 8, tt = rr % 8
            const int v = rr / ADJ_FLUSH, tt = rr % ADJ_FLUSH;
            const double *src = pbw + (v * ADJ_FLUSH + tt) * ADJ_ROW + half * 32;
            double s = 0.0;
#pragma unroll 8
            for (int q = 0; q < 32; ++q) s += src[q];
            s += __shfl_xor(s, 1);
            if (half == 0 && t0 + tt < t1) Qw[(w * 64 + t0 + tt) * 4 + v] = s;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (tid < nl) {
            const int l = lc + tid;
            double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
            for (int ww = 0; ww < nw; ++ww) {
                const double *qq = Qw + (ww * 64 + tid) * 4;
                q0 += qq[0];
                q1 += qq[1];
                q2 += qq[2];
                q3 += qq[3];
            }
            const double sg = ((l + k + m) & 1) ? -1.0 : 1.0;
            double2 g;
            if constexpr (BEAM) {
                double2 aa = coefs[(size_t)m * (2 * alm_lmax + 1 - m) / 2 + l];
                if (m == 0) aa.y = 0.0;
                g = cmul(make_double2(q0, -q1), aa);  // conj(Q+) a
                if (m > 0) {
                    const double2 t = cmul(make_double2(q2, q3), aa);  // Q- a
                    g.x += sg * t.x;
                    g.y -= sg * t.y;
                }
            } else {
                double2 bb = coefs[boff + l];
                if (k == 0) bb.y = 0.0;
                const double2 gp = cmul(make_double2(q0, q1), bb);
                if (m == 0) {
                    g = make_double2(gp.x, 0.0);
                } else {
                    const double2 gm = cmul(make_double2(q2, q3), bb);
                    g = make_double2(gp.x + sg * gm.x, gp.y - sg * gm.y);
                }
            }
            gk[l] = g;
        }
    }
}

// grad[i] = sum over slabs and m of GB[slab][m][i], in that fixed order, over the blm
// layout; the k = 0 column (entries i <= lmax) is real.
__global__ void k_reduce_over_m(const double2 *__restrict__ GB, double2 *__restrict__ grad, int64_t nblm, int lmax,
                                int nslab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nblm) return;
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < nslab * (lmax + 1); ++q) {
        const double2 v = GB[(size_t)q * nblm + i];
        s.x += v.x;
        s.y += v.y;
    }
    if (i <= lmax) s.y = 0.0;
    grad[i] = s;
}

// grad[i] = sum over slabs and k of GA[slab][k][i] in that fixed order (entries with
// k > l are zero).
__global__ void k_reduce_over_k(const double2 *__restrict__ GA, double2 *__restrict__ grad, int64_t nalm,
                                int kmax, int nslab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nalm) return;
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < nslab * (kmax + 1); ++q) {
        const double2 v = GA[(size_t)q * nalm + i];
        s.x += v.x;
        s.y += v.y;
    }
    grad[i] = s;
}

}  // namespace

// LDS bytes of an adjoint workgroup with nw waves.
static size_t adj_lds_bytes(int nw) {
    return sizeof(double) * (5 * 64 + (size_t)nw * 64 * 4 + (size_t)nw * 4 * ADJ_FLUSH * ADJ_ROW);
}

// Ring slabs per (k, m) column, northern rings per slab, waves per workgroup and
// rings per lane for the adjoint: a workgroup holds at most 1024 northern rings
// (8 waves, 32 rings per recursion and 4 per lane; its LDS fits one CU), so longer
// columns are split into equal slabs; per slab, the fewest idle ring slots.
static void adj_layout(int nring, int *rpt, int *nw, int *nslab, int *per) {
    const int nh = (nring + 1) / 2;
    const int ns = (nh + 1023) / 1024;
    const int pr = (nh + ns - 1) / ns;
    int best_r = 4, best_w = (pr + 127) / 128, best_waste = 1 << 30;
    for (int r = 4; r >= 1; --r) {
        const int waves = (pr + 32 * r - 1) / (32 * r);
        if (waves > 8 || adj_lds_bytes(waves) > 160 * 1024) continue;
        const int waste = waves * 32 * r - pr;
        if (waste < best_waste) {
            best_waste = waste;
            best_r = r;
            best_w = waves;
        }
    }
    *rpt = best_r;
    *nw = best_w;
    *nslab = ns;
    *per = pr;
}

int sc_adjoint_slabs(const sc_plan *p) { return ((p->nring + 1) / 2 + 1023) / 1024; }

#define SC_ADJ_CASE(R)                                                                                       \
    case R: {                                                                                                \
        auto kern = beam ? k_ring_sums_adjoint<R, true> : k_ring_sums_adjoint<R, false>;                      \
        e = sc_set_lds_attr((const void *)kern, lds);                                                        \
        if (e != hipSuccess) return e;                                                                       \
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(64 * nw), lds, p->stream, p->F, (const double2 *)coefs,    \
                           out, p->sbin_m, p->sbin_e, p->rtab, p->lmax, p->kmax, p->nring, p->alm_lmax, nslab, per); \
    } break;

static hipError_t ring_sums_adjoint(sc_plan *p, const double *coefs, double2 *out, bool beam) {
    int rpt, nw, nslab, per;
    adj_layout(p->nring, &rpt, &nw, &nslab, &per);
    const int nblk = (p->lmax + 1) * (p->kmax + 1) * nslab;
    const size_t lds = adj_lds_bytes(nw);
    hipError_t e = hipSuccess;
    switch (rpt) {
        SC_ADJ_CASE(1)
        SC_ADJ_CASE(2)
        SC_ADJ_CASE(3)
        default:
        SC_ADJ_CASE(4)
    }
    return hipGetLastError();
}

hipError_t sc_launch_ring_sums_adjoint(sc_plan *p, const double *blm, double *grad) {
    hipError_t e = ring_sums_adjoint(p, blm, p->GA, false);
    if (e != hipSuccess) return e;
    const int64_t nalm = (int64_t)(p->lmax + 1) * (p->lmax + 2) / 2;
    hipLaunchKernelGGL(k_reduce_over_k, dim3((unsigned)((nalm + 255) / 256)), dim3(256), 0, p->stream, p->GA,
                       (double2 *)grad, nalm, p->kmax, sc_adjoint_slabs(p));
    return hipGetLastError();
}

hipError_t sc_launch_ring_sums_adjoint_beam(sc_plan *p, const double *alm, double *grad) {
    hipError_t e = ring_sums_adjoint(p, alm, p->GB, true);
    if (e != hipSuccess) return e;
    const int64_t nblm = (int64_t)(p->kmax + 1) * (2 * p->lmax + 2 - p->kmax) / 2;
    hipLaunchKernelGGL(k_reduce_over_m, dim3((unsigned)((nblm + 255) / 256)), dim3(256), 0, p->stream, p->GB,
                       (double2 *)grad, nblm, p->lmax, sc_adjoint_slabs(p));
    return hipGetLastError();
}
