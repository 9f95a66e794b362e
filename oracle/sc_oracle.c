/*
 * sc_oracle.c -- plain CPU oracle for the spin-harmonic total convolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header or table with the HIP
 * library.
 *
 * What it computes (Galloway et al. 2022, "BeyondPlanck VIII", Sec. 2.1):
 *
 *   c(theta, phi, psi) = sum_{l, m_s, m_b} s_{l m_s} b*_{l m_b} [D^l_{m_s m_b}(phi, theta, psi)]*
 *
 * (the total-convolution sum, Eq. 2), with D^l_{mk}(a,b,g) = e^{-i m a} d^l_{mk}(b) e^{-i k g},
 * so that [D]* = e^{i m phi} d^l_{mk}(theta) e^{i k psi}.  The sum runs over every
 * l <= lmax, every |m| <= l and every |k| <= min(l, kmax): the coefficients with
 * negative orders are expanded from the stored m >= 0 / k >= 0 halves by the
 * real-field symmetry of Eq. 6 (b_{l,-k} = (-1)^k b*_{lk}, and the same for the
 * sky).  No pairing of +k/-k is used: the result is formed as a complex number
 * and its imaginary part is returned too, so a test can check that it vanishes.
 *
 * Wigner d^l_{mk}(theta): the standard (Condon-Shortley compatible) small
 * d-matrix.  For each (m, k) the column over l starts at l0 = max(|m|,|k|) from
 * the closed form of Wigner's explicit sum when one index equals +-l (a single
 * term survives), and continues with the three-term recursion in l
 *
 *   l sqrt(((l+1)^2-m^2)((l+1)^2-k^2)) d^{l+1}
 *       = (2l+1)(l(l+1)cos(theta) - m k) d^l - (l+1) sqrt((l^2-m^2)(l^2-k^2)) d^{l-1}
 *
 * evaluated in x87 long double (64-bit mantissa, exponent range to 1e+-4931),
 * which holds the smallest starting values (~1e-2900 at lmax 1024) without
 * any rescaling.  All sums are accumulated in long double.
 *
 * Everything is O(lmax^2 kmax) per sample.  It is slow on purpose.
 *
 * Coefficient layout (both arrays complex128, interleaved re/im):
 *   alm: index(l, m) = m (2 lmax + 1 - m) / 2 + l,   0 <= m <= l <= lmax
 *   blm: index(l, k) = k (2 lmax + 1 - k) / 2 + l,   0 <= k <= min(l, kmax)
 * Im(a_l0) and Im(b_l0) are ignored (real fields).
 * Pointings: float64 [n][3] = (theta, phi, psi), radians.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

static int iabs_(int x) { return x < 0 ? -x : x; }
static int imax_(int a, int b) { return a > b ? a : b; }

/* index of (l, m >= 0) in an lmax-triangular array */
static size_t tri_index(int lmax, int l, int m)
{
    return (size_t)m * (size_t)(2 * lmax + 1 - m) / 2 + (size_t)l;
}

/* a_{l,m} for any -l <= m <= l, from the stored m >= 0 half (real field). */
static void coef(const double *a, int lmax, int mmax, int l, int m, ld *re, ld *im)
{
    int am = iabs_(m);
    if (am > mmax || am > l) { *re = 0; *im = 0; return; }
    size_t i = tri_index(lmax, l, am);
    ld r = a[2 * i];
    ld q = (am == 0) ? 0.0L : (ld)a[2 * i + 1];
    if (m < 0) {
        /* a_{l,-m} = (-1)^m conj(a_{l,m}) */
        ld sg = (am & 1) ? -1.0L : 1.0L;
        *re = sg * r;
        *im = -sg * q;
    } else {
        *re = r;
        *im = q;
    }
}

/* sqrt(C(2l, l+n)) for |n| <= l, by the exact product formula of C(N, a). */
static ld sqrt_binom(int l, int n)
{
    int a = l + iabs_(n); /* C(2l, l+|n|) = C(2l, l-|n|) */
    ld c = 1.0L;
    /* each factor (a + i) / i is formed first, so the running product never exceeds
       C(2l, a) itself (about 1e4930 at l = 8192, inside the long double range) */
    for (int i = 1; i <= 2 * l - a; ++i) c *= (ld)(a + i) / (ld)i;
    return sqrtl(c);
}

static ld ipow_(ld x, int n) { return n == 0 ? 1.0L : powl(x, (ld)n); }

/*
 * d^{l0}_{m k}(theta) for l0 = max(|m|, |k|): Wigner's explicit sum collapses
 * to one term when one of the two orders is +-l0.
 *   d^l_{ l,k} = (-1)^{l-k} sqrt(C(2l,l+k)) c^{l+k} s^{l-k}
 *   d^l_{-l,k} =            sqrt(C(2l,l-k)) c^{l-k} s^{l+k}
 *   d^l_{m, l} =            sqrt(C(2l,l+m)) c^{l+m} s^{l-m}
 *   d^l_{m,-l} = (-1)^{l+m} sqrt(C(2l,l+m)) c^{l-m} s^{l+m}
 * with c = cos(theta/2), s = sin(theta/2).
 */
static ld d_start(int m, int k, ld c, ld s)
{
    int am = iabs_(m), ak = iabs_(k);
    if (am >= ak) {
        int l = am;
        if (m >= 0) {
            ld sg = ((l - k) & 1) ? -1.0L : 1.0L;
            return sg * sqrt_binom(l, k) * ipow_(c, l + k) * ipow_(s, l - k);
        }
        return sqrt_binom(l, k) * ipow_(c, l - k) * ipow_(s, l + k);
    }
    int l = ak;
    if (k > 0) return sqrt_binom(l, m) * ipow_(c, l + m) * ipow_(s, l - m);
    ld sg = ((l + m) & 1) ? -1.0L : 1.0L;
    return sg * sqrt_binom(l, m) * ipow_(c, l - m) * ipow_(s, l + m);
}

/* d[l] = d^l_{mk}(theta) for 0 <= l <= lmax (zero below l0), 0 <= theta <= pi/2. */
static void d_column_north(int lmax, int m, int k, ld theta, ld *d);

/* d[l] = d^l_{mk}(theta) for 0 <= l <= lmax (zero below l0).  Past the equator the
   column comes from d^l_{mk}(theta) = (-1)^{l+k} d^l_{-m,k}(pi - theta), so the
   recursion always runs at an angle whose 1 - cos is small near the nearer pole
   and keeps its full relative precision there. */
static void d_column(int lmax, int m, int k, ld theta, ld *d)
{
    const ld pi = 3.141592653589793238462643383279502884L;
    if (theta <= 0.5L * pi) {
        d_column_north(lmax, m, k, theta, d);
        return;
    }
    d_column_north(lmax, -m, k, pi - theta, d);
    for (int l = 0; l <= lmax; ++l)
        if ((l + k) & 1) d[l] = -d[l];
}

static void d_column_north(int lmax, int m, int k, ld theta, ld *d)
{
    int l0 = imax_(iabs_(m), iabs_(k));
    for (int l = 0; l <= lmax && l < l0; ++l) d[l] = 0.0L;
    if (l0 > lmax) return;
    ld c = cosl(0.5L * theta), s = sinl(0.5L * theta);
    /* 1 - cos(theta) = 2 sin^2(theta/2) at full relative precision: the coefficient
       l(l+1) cos(theta) - m k is evaluated as (l(l+1) - m k) - l(l+1) y, so near the
       poles the rounding of cos(theta) does not move the effective angle */
    ld y = 2.0L * s * s;
    ld dl = d_start(m, k, c, s), dm = 0.0L;
    d[l0] = dl;
    ld mm = (ld)m * m, kk = (ld)k * k, mk = (ld)m * k;
    for (int l = l0; l < lmax; ++l) {
        ld dn;
        if (l == 0) {
            dn = (1.0L - y) * dl; /* m = k = 0: d^1_00 = cos(theta) */
        } else {
            ld L = (ld)l, L1 = (ld)(l + 1);
            ld num1 = (2.0L * L + 1.0L) * ((L * L1 - mk) - L * L1 * y);
            ld num2 = L1 * sqrtl((L * L - mm) * (L * L - kk));
            ld den = L * sqrtl((L1 * L1 - mm) * (L1 * L1 - kk));
            dn = (num1 * dl - num2 * dm) / den;
        }
        dm = dl;
        dl = dn;
        d[l + 1] = dl;
    }
}

/*
 * out[((k + kmax) * (2 lmax + 1) + (m + lmax)) * (lmax + 1) + l] = d^l_{mk}(theta)
 * for |k| <= kmax, |m| <= lmax, 0 <= l <= lmax (zero where l < max(|m|,|k|)).
 */
int sco_wigner_d(int lmax, int kmax, double theta, double *out)
{
    if (lmax < 0 || kmax < 0 || kmax > lmax || !out) return -1;
    ld *d = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
    if (!d) return -2;
    for (int k = -kmax; k <= kmax; ++k)
        for (int m = -lmax; m <= lmax; ++m) {
            d_column(lmax, m, k, (ld)theta, d);
            double *o = out + ((size_t)(k + kmax) * (2 * lmax + 1) + (size_t)(m + lmax)) * (lmax + 1);
            for (int l = 0; l <= lmax; ++l) o[l] = (double)d[l];
        }
    free(d);
    return 0;
}

/* One sample of Eq. 2: the full triple sum, complex result. */
static void conv_sample(int lmax, int kmax, const double *alm, const double *blm,
                        ld theta, ld phi, ld psi, ld *d, ld *cre, ld *cim)
{
    ld sre = 0.0L, sim = 0.0L;
    for (int k = -kmax; k <= kmax; ++k) {
        for (int m = -lmax; m <= lmax; ++m) {
            int l0 = imax_(iabs_(m), iabs_(k));
            if (l0 > lmax) continue;
            d_column(lmax, m, k, theta, d);
            ld pre = 0.0L, pim = 0.0L; /* sum_l a_lm conj(b_lk) d^l_mk */
            for (int l = l0; l <= lmax; ++l) {
                ld ar, ai, br, bi;
                coef(alm, lmax, lmax, l, m, &ar, &ai);
                coef(blm, lmax, kmax, l, k, &br, &bi);
                pre += (ar * br + ai * bi) * d[l];
                pim += (ai * br - ar * bi) * d[l];
            }
            ld ang = (ld)m * phi + (ld)k * psi; /* [D]* = e^{i(m phi + k psi)} d */
            ld cs = cosl(ang), sn = sinl(ang);
            sre += pre * cs - pim * sn;
            sim += pre * sn + pim * cs;
        }
    }
    *cre = sre;
    *cim = sim;
}

/*
 * c_t for t < n.  out_re[t] = Re c_t, out_im[t] = Im c_t (zero up to rounding
 * for a real sky and beam; returned so that tests can check it).
 * nthreads <= 0 uses the OpenMP default.
 */
int sco_convolve(int lmax, int kmax, const double *alm, const double *blm,
                 const double *ptg, long n, double *out_re, double *out_im, int nthreads)
{
    if (lmax < 0 || kmax < 0 || kmax > lmax || n < 0) return -1;
    if (n == 0) return 0;
    if (!alm || !blm || !ptg || !out_re) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        ld *d = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        if (!d) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (long t = 0; t < n; ++t) {
                ld re, im;
                conv_sample(lmax, kmax, alm, blm, ptg[3 * t], ptg[3 * t + 1], ptg[3 * t + 2], d, &re, &im);
                out_re[t] = (double)re;
                if (out_im) out_im[t] = (double)im;
            }
            free(d);
        }
    }
    return err;
}

/*
 * Ring sums (the inner sum of Eq. 7 for one ring, before the azimuthal
 * synthesis):  F_k(theta_j, m) = sum_l a_lm conj(b_lk) d^l_mk(theta_j)
 * for 0 <= k <= kmax, |m| <= lmax.
 * F[((k * nth + j) * (2 lmax + 1) + (m + lmax)) * 2 + {0,1}] = (re, im).
 */
int sco_ring_sums(int lmax, int kmax, const double *alm, const double *blm,
                  const double *theta, long nth, double *F, int nthreads)
{
    if (lmax < 0 || kmax < 0 || kmax > lmax || nth < 0) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int err = 0;
    long ncol = (long)(kmax + 1) * nth;
#pragma omp parallel
    {
        ld *d = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        if (!d) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (long q = 0; q < ncol; ++q) {
                int k = (int)(q / nth);
                long j = q % nth;
                for (int m = -lmax; m <= lmax; ++m) {
                    double *o = F + (((size_t)k * nth + j) * (2 * lmax + 1) + (size_t)(m + lmax)) * 2;
                    int l0 = imax_(iabs_(m), k);
                    if (l0 > lmax) { o[0] = 0; o[1] = 0; continue; }
                    d_column(lmax, m, k, (ld)theta[j], d);
                    ld pre = 0.0L, pim = 0.0L;
                    for (int l = l0; l <= lmax; ++l) {
                        ld ar, ai, br, bi;
                        coef(alm, lmax, lmax, l, m, &ar, &ai);
                        coef(blm, lmax, kmax, l, k, &br, &bi);
                        pre += (ar * br + ai * bi) * d[l];
                        pim += (ai * br - ar * bi) * d[l];
                    }
                    o[0] = (double)pre;
                    o[1] = (double)pim;
                }
            }
            free(d);
        }
    }
    return err;
}

/*
 * Spin component maps at arbitrary points (Eq. 9 up to the spin-harmonic
 * sign convention):  T_k(theta, phi) = sum_{l, |m| <= l} a_lm conj(b_lk) d^l_mk(theta) e^{i m phi},
 * 0 <= k <= kmax.  T[(t * (kmax + 1) + k) * 2 + {0,1}].
 */
int sco_component_maps(int lmax, int kmax, const double *alm, const double *blm,
                       const double *theta, const double *phi, long n, double *T, int nthreads)
{
    if (lmax < 0 || kmax < 0 || kmax > lmax || n < 0) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        ld *d = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        if (!d) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (long t = 0; t < n; ++t) {
                for (int k = 0; k <= kmax; ++k) {
                    ld tre = 0.0L, tim = 0.0L;
                    for (int m = -lmax; m <= lmax; ++m) {
                        int l0 = imax_(iabs_(m), k);
                        if (l0 > lmax) continue;
                        d_column(lmax, m, k, (ld)theta[t], d);
                        ld pre = 0.0L, pim = 0.0L;
                        for (int l = l0; l <= lmax; ++l) {
                            ld ar, ai, br, bi;
                            coef(alm, lmax, lmax, l, m, &ar, &ai);
                            coef(blm, lmax, kmax, l, k, &br, &bi);
                            pre += (ar * br + ai * bi) * d[l];
                            pim += (ai * br - ar * bi) * d[l];
                        }
                        ld ang = (ld)m * (ld)phi[t];
                        ld cs = cosl(ang), sn = sinl(ang);
                        tre += pre * cs - pim * sn;
                        tim += pre * sn + pim * cs;
                    }
                    T[((size_t)t * (kmax + 1) + k) * 2] = (double)tre;
                    T[((size_t)t * (kmax + 1) + k) * 2 + 1] = (double)tim;
                }
            }
            free(d);
        }
    }
    return err;
}

/*
 * Adjoint of the convolution with respect to the stored sky coefficients.
 * The convolution is real-linear in (Re a_lm, Im a_lm) for m > 0 and in
 * Re a_l0.  For L = sum_t y_t c_t this returns
 *     g_lm = dL/dRe(a_lm) + i dL/dIm(a_lm)
 * (zero imaginary part for m = 0), written out from the derivative of the
 * full sum of Eq. 2:  with X_lm(t) = e^{i m phi} sum_{|k|<=kmax} conj(b_lk) d^l_mk(theta) e^{i k psi},
 *   d c_t / d Re a_lm = Re[X_lm + (-1)^m X_{l,-m}],
 *   d c_t / d Im a_lm = Re[i X_lm - i (-1)^m X_{l,-m}]      (m > 0),
 *   d c_t / d Re a_l0 = Re X_l0.
 * grad is complex128 in the alm layout.
 */
int sco_adjoint(int lmax, int kmax, const double *blm, const double *ptg,
                const double *y, long n, double *grad, int nthreads)
{
    if (lmax < 0 || kmax < 0 || kmax > lmax || n < 0) return -1;
    size_t nalm = tri_index(lmax, lmax, lmax) + 1;
    memset(grad, 0, sizeof(double) * 2 * nalm);
    if (n == 0) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        ld *d = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        /* X[(m + lmax) * (lmax + 1) + l], complex */
        ld *X = (ld *)malloc(sizeof(ld) * 2 * (size_t)(2 * lmax + 1) * (lmax + 1));
        ld *acc = (ld *)calloc(2 * nalm, sizeof(ld));
        if (!d || !X || !acc) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (long t = 0; t < n; ++t) {
                ld th = ptg[3 * t], ph = ptg[3 * t + 1], ps = ptg[3 * t + 2];
                memset(X, 0, sizeof(ld) * 2 * (size_t)(2 * lmax + 1) * (lmax + 1));
                for (int k = -kmax; k <= kmax; ++k)
                    for (int m = -lmax; m <= lmax; ++m) {
                        int l0 = imax_(iabs_(m), iabs_(k));
                        if (l0 > lmax) continue;
                        d_column(lmax, m, k, th, d);
                        ld ang = (ld)m * ph + (ld)k * ps;
                        ld cs = cosl(ang), sn = sinl(ang);
                        for (int l = l0; l <= lmax; ++l) {
                            ld br, bi;
                            coef(blm, lmax, kmax, l, k, &br, &bi);
                            /* conj(b) d e^{i ang} */
                            ld pr = br * d[l], pi = -bi * d[l];
                            ld *x = X + 2 * ((size_t)(m + lmax) * (lmax + 1) + l);
                            x[0] += pr * cs - pi * sn;
                            x[1] += pr * sn + pi * cs;
                        }
                    }
                ld yt = y[t];
                for (int l = 0; l <= lmax; ++l)
                    for (int m = 0; m <= l; ++m) {
                        size_t i = tri_index(lmax, l, m);
                        ld *xp = X + 2 * ((size_t)(m + lmax) * (lmax + 1) + l);
                        if (m == 0) {
                            acc[2 * i] += yt * xp[0];
                            continue;
                        }
                        ld *xn = X + 2 * ((size_t)(-m + lmax) * (lmax + 1) + l);
                        ld sg = (m & 1) ? -1.0L : 1.0L;
                        ld dre = xp[0] + sg * xn[0];     /* Re[X + (-1)^m X-] */
                        ld dim = -xp[1] + sg * xn[1];    /* Re[i X - i (-1)^m X-] */
                        acc[2 * i] += yt * dre;
                        acc[2 * i + 1] += yt * dim;
                    }
            }
#pragma omp critical
            {
                for (size_t i = 0; i < 2 * nalm; ++i) grad[i] += (double)acc[i];
            }
        }
        free(d);
        free(X);
        free(acc);
    }
    return err;
}
