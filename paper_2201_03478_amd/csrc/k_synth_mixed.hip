// k_synth_mixed.hip -- ring sums with the contraction on the matrix cores (the
// precision variant).
//
// Same quantity as k_synth.hip (the inner sums of Eqs. 7/9, Galloway et al.
// 2022, Sec. 2.1, for both signs of m):
//     F_k(theta_j, m) = sum_l a_lm conj(b_lk) d^l_mk(theta_j),
// from the same FP64 recursions: extended-exponent start values, the normalised
// three-term recursion in l on northern rings for the columns (m, k) and
// (-m, k) (k_synth.hip explains the layout and the reflection that gives the
// southern rings).  What changes is the contraction of the d values with the
// coefficient products: instead of four FP64 FMAs per d value on the VALU it runs
// as v_mfma_f32_4x4x1_16b_f32, 16 independent 4x4 outer products per wave:
// lane 4b + i supplies its ring's u^l rounded to FP32 (row i of block b), lane
// 4b + j the FP32 weight component j of the step (Re wp, Im wp, Re wm, Im wm;
// the same for R+ and the sign-alternated R-, as in k_synth.hip), and register i
// of lane 4b + j accumulates component j of ring 4b + i in FP32.  Every 64 steps
// the FP32 accumulators are added into FP64 sums and cleared, so FP32 rounding
// enters only through the products and 64-term partial sums.  The VALU keeps the
// recursion (two FP64 FMAs per d value) and one conversion.
//
// The recursion stays in FP64: on this chip an unpacked FP32 FMA costs what an
// FP64 FMA costs, and an FP32 recursion drifts by ~1e-6 relative by l ~ 1000,
// more than the error budget of the form.  While a ring's values are still scaled
// (extended exponent e < 0, true |d| < 2^-600) it feeds zero to the matrix cores.
#include "wigner_rec.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

using namespace wrec;

struct MxCoef {
    double a, b;
    float w;
};

__device__ __forceinline__ MxCoef mx_load(int t, const double *cA, const double *cB, const float *cW) {
    // cB points at the lane's half of [tp][64]; cW at its component (entry (t, j) at 4 t + j)
    return MxCoef{cA[t], cB[t], cW[4 * t]};
}

template <int RPT, bool MASK>
__device__ __forceinline__ void mx_step(const MxCoef &c, const double *x, double *u, double *up, const int *e,
                                        floatx4 *acc) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        float v = (float)u[r];
        if (MASK && e[r] != 0) v = 0.f;  // scaled value: below 2^-600 in true units
        acc[r] = __builtin_amdgcn_mfma_f32_4x4x1f32(v, c.w, acc[r], 0, 0, 0);
        const double un = fma(fma(c.a, x[r], c.b), u[r], -up[r]);  // x holds y' = -+(1 - cos(theta))
        up[r] = u[r];
        u[r] = un;
    }
}

// Steps t0 .. t1-1 with the coefficient lookahead of k_synth.hip.
template <int RPT, bool MASK>
__device__ __forceinline__ void mx_steps(int t0, int t1, const double *cA, const double *cB, const float *cW,
                                         const double *x, double *u, double *up, const int *e, floatx4 *acc) {
    const int te = t0 + ((t1 - t0) & ~3);
    if (te > t0) {
        MxCoef a0 = mx_load(t0, cA, cB, cW), a1 = mx_load(t0 + 1, cA, cB, cW);
        for (int t = t0; t < te; t += 4) {
            const MxCoef b0 = mx_load(t + 2, cA, cB, cW), b1 = mx_load(t + 3, cA, cB, cW);
            __builtin_amdgcn_sched_barrier(0);
            mx_step<RPT, MASK>(a0, x, u, up, e, acc);
            mx_step<RPT, MASK>(a1, x, u, up, e, acc);
            const int tn = t + 4 < te ? t + 4 : t;  // last iteration: harmless re-read
            a0 = mx_load(tn, cA, cB, cW);
            a1 = mx_load(tn + 1, cA, cB, cW);
            __builtin_amdgcn_sched_barrier(0);
            mx_step<RPT, MASK>(b0, x, u, up, e, acc);
            mx_step<RPT, MASK>(b1, x, u, up, e, acc);
        }
    }
    for (int t = te; t < t1; ++t) mx_step<RPT, MASK>(mx_load(t, cA, cB, cW), x, u, up, e, acc);
}

template <int RPT, typename FT, bool TAB>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RPT <= 3 ? 3 : 2)))
k_ring_sums_mixed(const double2 *__restrict__ alm, const double2 *__restrict__ blm, FT *__restrict__ F,
                  const double *__restrict__ sbin_m, const int *__restrict__ sbin_e,
                  const double *__restrict__ rtab, const double2 *__restrict__ rroot,
                  const double4 *__restrict__ ctab, const long long *__restrict__ ctab_off, int lmax, int kmax,
                  int nring, int ngroups, int alm_lmax) {
    __shared__ double cA[64], cB[2 * 64];
    __shared__ float cW[64 * 4];
    __shared__ double Fs[RPT][64][4];

    int b, g;  // b = column m (kmax + 1) + k
    xcd_column_group(blockIdx.x, (lmax + 1) * (kmax + 1), ngroups, b, g);
    const int k = b % (kmax + 1);
    const int m = b / (kmax + 1);
    const int lane = threadIdx.x;
    const int tp = lane >> 5, sub = lane & 31;  // recursion R+ (0) or R- (1); northern ring slot
    const int l0 = m > k ? m : k;
    const int mn = m < k ? m : k;
    const int nm = 2 * lmax + 1;
    const int nh = (nring + 1) / 2;

    double x[RPT], u[RPT], up[RPT];
    int e[RPT];
    floatx4 acc[RPT];
    double sacc[RPT][4];  // FP64 sums of acc: component lane % 4 of ring (lane & ~3) + i

    const XN pref = {sbin_m[l0 * (kmax + 1) + mn], sbin_e[l0 * (kmax + 1) + mn]};
    const double pfe = (double)pref.e, pfm = log2(pref.m);
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 32 + sub;
        const bool on = j < nh && (tp == 0 || (m > 0 && j != nring - 1 - j));
        acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) sacc[r][i] = 0.0;
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

    const size_t aoff = (size_t)m * (2 * alm_lmax + 1 - m) / 2;
    const size_t boff = (size_t)k * (2 * lmax + 1 - k) / 2;
    double s_prev = 1.0, s_cur = 1.0;
    const double *cBt = cB + 64 * tp;
    const float *cWt = cW + (lane & 3);
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
            // (Re, Im) of wp, then of wm, rounded to FP32
            if (which < 2) {
                float *w = cW + 4 * lane + 2 * which;
                w[0] = (float)v.x;
                w[1] = (float)v.y;
            }
        });
        __syncthreads();
        if (TAB) cnext = chunk_coefs_tab(ccol, lc + 64, lane, l0, lmax);  // in flight during the steps
        const int nl = (lmax - lc + 1) < 64 ? (lmax - lc + 1) : 64;
        if (fast) {
            mx_steps<RPT, false>(0, nl, cA, cBt, cWt, x, u, up, e, acc);
        } else {
            // rescaling checked once per 32 steps (see k_synth.hip); scaled rings feed zero
            for (int t0 = 0; t0 < nl; t0 += 32) {
                const int t1 = t0 + 32 < nl ? t0 + 32 : nl;
                if (fast)
                    mx_steps<RPT, false>(t0, t1, cA, cBt, cWt, x, u, up, e, acc);
                else
                    mx_steps<RPT, true>(t0, t1, cA, cBt, cWt, x, u, up, e, acc);
                if (fast) continue;
                bool low = false;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    if (fabs(u[r]) > REC_BIG) {
                        u[r] = rec_down(u[r]);
                        up[r] = rec_down(up[r]);
                        e[r] += 1;
                    }
                    low |= e[r] != 0;
                }
                fast = !__any(low);
            }
        }
        // 64-step partial sums into FP64
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sacc[r][i] += (double)acc[r][i];
            acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    }

    // lane 4q + c holds component c of rings 4q + i in sacc[.][i]: regroup per ring
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) Fs[r][(lane & ~3) + i][lane & 3] = sacc[r][i];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = (g * RPT + r) * 32 + sub;
        const int js = nring - 1 - j;
        const double *f = Fs[r][lane];
        const double2 fp = make_double2(f[0], f[1]), fm = make_double2(f[2], f[3]);
        if (j < nh) {
            if (tp == 0) {
                st2(&F[((size_t)k * nm + (m + lmax)) * nring + j], fp);
                if (m > 0 || js != j) st2(&F[((size_t)k * nm + (lmax - m)) * nring + js], fm);
            } else if (m > 0 && js != j) {  // exchanged, times (-1)^k (see k_synth.hip)
                const double sk = (k & 1) ? -1.0 : 1.0;
                st2(&F[((size_t)k * nm + (lmax - m)) * nring + j], cscale(fm, sk));
                st2(&F[((size_t)k * nm + (m + lmax)) * nring + js], cscale(fp, sk));
            }
        }
    }
}

}  // namespace

template <typename FT, bool TAB>
static void launch_mixed(sc_plan *p, const double *alm, const double *blm, FT *F) {
    const int nblk = (p->lmax + 1) * (p->kmax + 1) * p->ngroups_mx;
    auto kern = k_ring_sums_mixed<4, FT, TAB>;
    switch (p->rpt_mx) {
        case 1: kern = k_ring_sums_mixed<1, FT, TAB>; break;
        case 2: kern = k_ring_sums_mixed<2, FT, TAB>; break;
        case 3: kern = k_ring_sums_mixed<3, FT, TAB>; break;
        default: break;
    }
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(64), 0, p->stream, (const double2 *)alm, (const double2 *)blm, F,
                       p->sbin_m, p->sbin_e, p->rtab, p->rroot, p->ctab, p->ctab_off, p->lmax, p->kmax, p->nring,
                       p->ngroups_mx, p->alm_lmax);
}

hipError_t sc_launch_ring_sums_mixed(sc_plan *p, const double *alm, const double *blm) {
    if (p->mid32) {
        if (p->ctab)
            launch_mixed<float2, true>(p, alm, blm, (float2 *)p->F);
        else
            launch_mixed<float2, false>(p, alm, blm, (float2 *)p->F);
    } else {
        if (p->ctab)
            launch_mixed<double2, true>(p, alm, blm, p->F);
        else
            launch_mixed<double2, false>(p, alm, blm, p->F);
    }
    return hipGetLastError();
}

// The same layout as the FP64 kernel (32 northern rings per recursion and lane slot).
void sc_choose_ring_layout_mixed(int nring, int *rpt, int *ngroups) { sc_choose_ring_layout(nring, rpt, ngroups); }
