/*
 * sanitize_check.c -- test infrastructure: runs every entry point of the oracle
 * (sc_oracle.c) on small seeded inputs, including lmax 0, kmax = lmax, the poles,
 * phi = 2 pi and negative psi, and checks the argument errors.  It is built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py, so
 * an out-of-bounds access, use of freed memory, leak, signed overflow or invalid
 * shift anywhere in the oracle ends the run with an error.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int sco_wigner_d(int lmax, int kmax, double theta, double *out);
int sco_convolve(int lmax, int kmax, const double *alm, const double *blm, const double *ptg, long n,
                 double *out_re, double *out_im, int nthreads);
int sco_ring_sums(int lmax, int kmax, const double *alm, const double *blm, const double *theta, long nth,
                  double *F, int nthreads);
int sco_component_maps(int lmax, int kmax, const double *alm, const double *blm, const double *theta,
                       const double *phi, long n, double *T, int nthreads);
int sco_adjoint(int lmax, int kmax, const double *blm, const double *ptg, const double *y, long n, double *grad,
                int nthreads);

static unsigned state = 12345u;
static double urand(void) {
    state = state * 1664525u + 1013904223u;
    return (double)(state >> 8) / 16777216.0;
}

static double *vec(size_t n) {
    double *v = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) v[i] = 2.0 * urand() - 1.0;
    return v;
}

static int fails = 0;
static void expect(int got, int want, const char *what, int L, int K) {
    if (got != want) {
        printf("%s (lmax %d, kmax %d): returned %d, expected %d\n", what, L, K, got, want);
        ++fails;
    }
}

int main(void) {
    const double pi = 3.14159265358979323846;
    const int cases[][2] = {{0, 0}, {1, 1}, {7, 3}, {16, 16}, {40, 5}};
    for (size_t c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c) {
        const int L = cases[c][0], K = cases[c][1];
        const size_t nalm = (size_t)(L + 1) * (L + 2) / 2;
        const size_t nblm = (size_t)(K + 1) * (L + 1) - (size_t)K * (K + 1) / 2;
        double *alm = vec(2 * nalm), *blm = vec(2 * nblm);
        const long n = 9;
        double ptg[27] = {0.0, 0.3, 1.0, pi, 2.0, -0.5, 1e-9, 2.0 * pi, 3.0, pi - 1e-9, 0.0, 6.28,
                          0.7, 1.1, 2.2, 1.9, 4.0, 0.1, 2.5, 5.5, -3.0, 0.2, 0.01, 0.02, 3.0, 3.1, 3.2};
        double *wd = vec((size_t)(2 * K + 1) * (2 * L + 1) * (L + 1));
        const double thetas[3] = {0.3, 0.0, pi};
        for (int t = 0; t < 3; ++t) expect(sco_wigner_d(L, K, thetas[t], wd), 0, "sco_wigner_d", L, K);
        double *re = vec(n), *im = vec(n);
        expect(sco_convolve(L, K, alm, blm, ptg, n, re, im, 2), 0, "sco_convolve", L, K);
        const long nth = 5;
        const double th[5] = {0.0, 0.1, pi / 2, 3.0, pi};
        double *F = vec((size_t)(K + 1) * nth * (2 * L + 1) * 2);
        expect(sco_ring_sums(L, K, alm, blm, th, nth, F, 2), 0, "sco_ring_sums", L, K);
        double phi[5] = {0.0, 1.0, 2.0 * pi, -1.0, 3.0};
        double *T = vec((size_t)nth * (K + 1) * 2);
        expect(sco_component_maps(L, K, alm, blm, th, phi, nth, T, 2), 0, "sco_component_maps", L, K);
        double *y = vec(n), *g = vec(2 * nalm);
        expect(sco_adjoint(L, K, blm, ptg, y, n, g, 2), 0, "sco_adjoint", L, K);
        for (size_t i = 0; i < (size_t)n; ++i)
            if (!isfinite(re[i]) || !isfinite(im[i])) {
                printf("non-finite convolution at lmax %d, kmax %d, sample %zu\n", L, K, i);
                ++fails;
            }
        free(alm); free(blm); free(wd); free(re); free(im); free(F); free(T); free(y); free(g);
    }
    /* argument errors */
    double dummy[8] = {0};
    expect(sco_convolve(-1, 0, dummy, dummy, dummy, 1, dummy, dummy, 1), -1, "sco_convolve lmax < 0", -1, 0);
    expect(sco_convolve(3, 4, dummy, dummy, dummy, 1, dummy, dummy, 1), -1, "sco_convolve kmax > lmax", 3, 4);
    expect(sco_adjoint(2, 0, dummy, dummy, dummy, -1, dummy, 1), -1, "sco_adjoint n < 0", 2, 0);
    if (fails) return 1;
    printf("oracle entry points ran clean\n");
    return 0;
}
