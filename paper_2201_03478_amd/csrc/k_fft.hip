// k_fft.hip -- theta upsampling and phi synthesis of the component maps.
//
// After the ring sums F_k(theta_j, m) = sum_l a_lm conj(b_lk) d^l_mk(theta_j)
// (the inner sums of Eqs. 7/9 of Galloway et al. 2022, Sec. 2.1, on rings
// theta_j = (j + 1/2) pi / nring), each spin-k map T_k(theta, phi) =
// sum_m F_k(theta, m) e^{i m phi} is brought onto an oversampled equiangular
// grid ready for interpolation (the finite-resolution cube of Sec. 2.1):
//
//  theta: F_k(., m) is a trigonometric polynomial of degree <= lmax in theta
//    whose continuation to the full circle obeys F(-theta) = (-1)^{m-k} F(theta)
//    (from d^l_mk(-theta) = (-1)^{m-k} d^l_mk(theta)).  A length-2 nring FFT of
//    the extended column gives its Fourier coefficients exactly; they are
//    divided by the interpolation kernel's transform (theta and phi factors),
//    zero-padded and inverse-transformed onto theta_r = r 2 pi / n2os, keeping
//    rows r in [-W/2 + 1, n2os/2 + W/2] (ghost rows past the poles included).
//  phi: per (k, row) the deconvolved m-spectrum is inverse-transformed onto
//    phi_q = q 2 pi / nphi, q in [-W/2 + 1, nphi + W/2 - 1] (wrap copies), and
//    stored as the real components M_0 = T_0, M_1 = 0, M_{2k} = 2 Re T_k,
//    M_{2k+1} = -2 Im T_k, so that c = sum_c basis_c(psi) M_c (Eq. 8) with
//    basis_{2k} = cos k psi and basis_{2k+1} = sin k psi.
#include "fft_lds.h"

namespace {

// one aligned store of a component pair (the padded row length is even)
template <typename T>
__device__ inline void store_pair(T *o, double a, double b);
template <>
__device__ inline void store_pair<double>(double *o, double a, double b) {
    *(double2 *)o = make_double2(a, b);
}
template <>
__device__ inline void store_pair<float>(float *o, double a, double b) {
    *(float2 *)o = make_float2((float)a, (float)b);
}

// two adjacent component pairs as one aligned 16-byte store (FP32 maps)
template <typename T>
__device__ inline void store_quad(T *o, T a, T b, T c, T d);
template <>
__device__ inline void store_quad<float>(float *o, float a, float b, float c, float d) {
    *(float4 *)o = make_float4(a, b, c, d);
}
template <>
__device__ inline void store_quad<double>(double *o, double a, double b, double c, double d) {
    ((double2 *)o)[0] = make_double2(a, b);
    ((double2 *)o)[1] = make_double2(c, d);
}

// Two columns per workgroup.  Columns mi and mi + 1 (same k) have opposite
// parities s1 = (-1)^{m-k} and s2 = -s1, and for an extended column with
// f(n2 - 1 - j) = s f(j) the transform obeys X(-n) = s w^n X(n), w = e^{-2 pi i / n2}.
// So one transform of h = f1 + i f2 gives both: with H = FFT(h),
// X1 = (H(n) + s1 w^{-n} H(-n)) / 2 and X2 = (H(n) - s1 w^{-n} H(-n)) / (2 i).
// The deconvolution factor is p(n) d(m), p(n) = e^{-i pi n / n2} q(|n|) with q real,
// so p(n) w^{-n} = conj(p(n)), and the combined spectrum Y1 + i Y2 is
//     Z(n) = a p(n) H(n) + b conj(p(n)) H(-n),  a = (d1 + d2) / 2,  b = s1 (d1 - d2) / 2.
// The upsampled columns keep the parities, G_c(-r) = s_c G_c(r), so the inverse
// transform of Z, O = G1 + i G2, separates as G1 = (O(r) + s1 O(-r)) / 2 and
// G2 = (O(r) - s1 O(-r)) / (2 i) (the halves are folded into a and b).  For odd
// nm the last column is alone (f2 = 0, d2 = d1 makes Z = d1 p H).
//
// F and G are complex128 or complex64 (FT, GT); G rows have stride gst.  With
// compile-time transforms (TWL) the passes take their twiddles from LDS bases that
// the workgroup loads first, so no pass waits for a global load.  (A persistent
// variant that walks consecutive pairs and prefetches the next pair's columns
// measured slower at lmax 512 than one pair per workgroup.)
template <int NT, int PT, typename S2, typename SOS, typename FT, typename GT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    FftLen<S2>::value > 0 && FftLen<SOS>::value > 0 && sizeof(GT) == sizeof(float2) ? (NT > 256 ? 5 : 6) : 4)))
k_theta_upsample(const FT *__restrict__ F, GT *__restrict__ G, int lmax, int nring, int rows, int gst,
                 int W, FftPlan P2, FftPlan Pos, const double2 *__restrict__ tw2,
                 const double2 *__restrict__ twos, const double2 *__restrict__ phase,
                 const double *__restrict__ dphi) {
    using Fwd = FftRun<-1, NT, PT, S2>;
    using Inv = FftRun<1, NT, PT, SOS>;
    constexpr bool TWL = FftLen<S2>::value > 0 && FftLen<SOS>::value > 0;
    // complex64 spectra with compile-time transforms: the transform buffer holds
    // complex64 too (half the LDS per workgroup); the arithmetic stays FP64
    using BT = typename std::conditional<TWL && sizeof(GT) == sizeof(float2), float2, double2>::type;
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int npair = lmax + 1;  // ceil(nm / 2)
    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // consecutive column pairs share an XCD
    const int k = blk / npair;
    const int mi = 2 * (blk - k * npair);
    const bool two = mi + 1 < nm;
    const int m = mi - lmax;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int n2 = P2.n, nos = Pos.n;
    BT *B = (BT *)sbuf;                         // length nos; the forward transform runs in B[0 .. n2)
    double2 *T2 = (double2 *)(B + nos);  // LDS twiddle bases (TWL): forward, then inverse (nos is even)
    // With a complex64 buffer of nos >= 2 n2 points the forward transform still fits
    // in complex128 (the same bytes): it runs without conversions, and only the
    // deconvolved spectrum is stored in complex64 for the inverse transform.
    using FT2 = typename std::conditional<(TWL && sizeof(BT) == sizeof(float2) &&
                                           FftLen<SOS>::value >= 2 * FftLen<S2>::value), double2, BT>::type;
    FT2 *Bf = (FT2 *)sbuf;
    double2 *Tos = T2;
    if constexpr (TWL) {
        Tos = T2 + Fwd::ntw;
        Fwd::load_tw(T2, tw2, tid);
        Inv::load_tw(Tos, twos, tid);  // visible after the fill's barrier
    }

    const double s1 = ((m - k) & 1) ? -1.0 : 1.0;
    const FT *col = F + ((size_t)k * nm + mi) * nring;
    for (int j = tid; j < nring; j += nth) {
        const double2 a = ld2(col + j);
        const double2 b = two ? ld2(col + nring + j) : make_double2(0.0, 0.0);
        st2(Bf + j, make_double2(a.x - b.y, a.y + b.x));                         // a + i b
        st2(Bf + n2 - 1 - j, make_double2(s1 * (a.x + b.y), s1 * (a.y - b.x)));  // s1 (a - i b)
    }
    __syncthreads();
    if constexpr (TWL)
        Fwd::run_l(Bf, T2, tid);
    else
        Fwd::run((double2 *)B, P2, tw2, tid, nth);

    // Coefficients n in [-lmax, lmax]: n >= 0 stay at n, n < 0 move from
    // n + n2 to n + nos (sources and targets are disjoint since nos >= n2 + lmax),
    // everything in between becomes zero.  nm < n2 <= nos / 2 <= NT PT / 2, so
    // each thread holds at most ceil(PT / 2) coefficients.
    constexpr int MAXC = (PT + 1) / 2;
    const double d1 = dphi[m < 0 ? -m : m];
    const double d2 = two ? dphi[m + 1 < 0 ? -(m + 1) : m + 1] : d1;
    const double ca = 0.25 * (d1 + d2), cb = 0.25 * s1 * (d1 - d2);
    double2 xs[MAXC];
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * nth;
        if (t < nm) {
            const int n = t - lmax;
            const double2 p = phase[t];
            const double2 hp = ld2(Bf + (n < 0 ? n + n2 : n)), hm = ld2(Bf + (n > 0 ? n2 - n : -n));
            const double2 u = cmul(p, hp), v = cmul(cconj(p), hm);
            xs[i] = make_double2(ca * u.x + cb * v.x, ca * u.y + cb * v.y);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * nth;
        if (t < nm) {
            const int n = t - lmax;
            st2(B + (n < 0 ? n + nos : n), xs[i]);
        }
    }
    for (int t = lmax + 1 + tid; t < nos - lmax; t += nth) st2(B + t, make_double2(0.0, 0.0));
    __syncthreads();
    if constexpr (TWL)
        Inv::run_l(B, Tos, tid);
    else
        Inv::run((double2 *)B, Pos, twos, tid, nth);

    const int r0 = -W / 2 + 1;
    GT *gk = G + (size_t)k * rows * gst + mi;
    if constexpr (sizeof(GT) == sizeof(float2)) {
        // complex64: one thread writes both columns of a row as one 16-byte store (gst
        // and mi are even; an odd last column is written with a zero beside it, in the
        // padding element of the row)
        for (int row = tid; row < rows; row += nth) {
            int r = row + r0;
            r = r < 0 ? r + nos : (r >= nos ? r - nos : r);
            const int rm = r == 0 ? 0 : nos - r;
            const double2 o = ld2(B + r), om = ld2(B + rm);
            const double2 g1 = make_double2(o.x + s1 * om.x, o.y + s1 * om.y);
            const double2 g2 = two ? make_double2(o.y - s1 * om.y, s1 * om.x - o.x) : make_double2(0.0, 0.0);
            *(float4 *)(gk + (size_t)row * gst) = make_float4((float)g1.x, (float)g1.y, (float)g2.x, (float)g2.y);
        }
    } else {
        // Lane pairs write the two columns of a row side by side (one 32-byte run).
        for (int q = tid; q < 2 * rows; q += nth) {
            const int row = q >> 1, c = q & 1;
            if (c && !two) continue;
            int r = row + r0;
            r = r < 0 ? r + nos : (r >= nos ? r - nos : r);
            const int rm = r == 0 ? 0 : nos - r;
            const double2 o = ld2(B + r), om = ld2(B + rm);
            const double2 g = c == 0 ? make_double2(o.x + s1 * om.x, o.y + s1 * om.y)
                                     : make_double2(o.y - s1 * om.y, s1 * om.x - o.x);  // -i (o - s1 om)
            gk[(size_t)row * gst + c] = g;
        }
    }
}

// Map values of one k at one column, (M_{2k}, M_{2k+1}) = (2 Re T_k, -2 Im T_k) or (Re T_0, 0).
__device__ __forceinline__ double2 phi_pair(double2 v, int k) {
    return k == 0 ? make_double2(v.x, 0.0) : make_double2(2.0 * v.x, -2.0 * v.y);
}

// G row (nm spectral values) into registers; lanes past nm read a valid duplicate,
// which phi_scatter replaces by zero.
template <int NT, int MAXC, typename GT>
__device__ __forceinline__ void phi_load(GT (&spec)[MAXC], const GT *__restrict__ src, int tid, int nm) {
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * NT;
        spec[i] = src[t < nm ? t : nm - 1];
    }
}

// Zero-padded spectrum in A: m >= 0 at m, m < 0 at m + np, zeros in between (lanes
// past nm write a zero into that band too).
template <int NT, int MAXC, typename BT, typename GT>
__device__ __forceinline__ void phi_scatter(BT *A, const GT (&spec)[MAXC], int tid, int lmax, int np) {
    const int nm = 2 * lmax + 1;
    for (int t = lmax + 1 + tid; t < np - lmax; t += NT) st2(A + t, make_double2(0.0, 0.0));
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * NT;
        const int m = t - lmax;
        const bool in = t < nm;
        const double2 v = make_double2((double)spec[i].x, (double)spec[i].y);
        st2(A + (in ? (m < 0 ? m + np : m) : lmax + 1), make_double2(in ? v.x : 0.0, in ? v.y : 0.0));
    }
}

// One workgroup per (row, group of KP = 1 or 2 consecutive k).  With KP = 2 the two
// transforms run one after the other in one LDS buffer: the second k's spectrum is
// loaded into registers while the first is transformed, and the first k's columns
// wait in registers, so each lane writes both k's component pairs of a column as
// one 16-byte store.  In the column-tiled maps (FP32: four components, FP64: the
// pair of one k per 16-byte group) the workgroup's stores of eight consecutive
// columns fill one 128-byte line.
template <typename T, int NT, int PT, typename SP, int KP, typename GT>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(FftLen<SP>::value > 0 && sizeof(GT) == sizeof(float2) && NT <= 256 ? 5 : 4)))
k_phi_synthesis(const GT *__restrict__ G, T *__restrict__ maps, int lmax, int rows, int gst, int cols, int ncp,
                int W, int nk, FftPlan Pp, const double2 *__restrict__ twp) {
    static_assert(KP == 1 || KP == 2, "one or two k per workgroup");
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int ngrp = (nk + KP - 1) / KP;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // consecutive k groups of one row share an XCD
    const int row = blk / ngrp;
    const int k0 = (blk - row * ngrp) * KP;
    const bool two = KP == 2 && k0 + 1 < nk;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int np = Pp.n;
    constexpr int NP = FftLen<SP>::value;  // 0: runtime-planned transform
    // complex64 spectra with a compile-time transform: complex64 transform buffer
    // (half the LDS per workgroup), FP64 arithmetic
    using BT = typename std::conditional<(NP > 0 && sizeof(GT) == sizeof(float2)), float2, double2>::type;
    BT *A = (BT *)sbuf;
    using Run = FftRun<1, NT, PT, SP>;
    double2 *Tw = (double2 *)(A + np);  // compile-time transforms: LDS twiddle bases (np is even)
    if constexpr (NP > 0) Run::load_tw(Tw, twp, tid);  // visible after the first barrier
    constexpr int MAXC = (PT + 1) / 2;                            // nm <= NT MAXC
    constexpr int MAXS = NP > 0 ? (NP + 15 + NT - 1) / NT : PT + 1;  // cols <= np + 15 <= NT MAXS
    const int q0 = -W / 2 + 1;
    const GT *src = G + ((size_t)k0 * rows + row) * gst;
    GT spec[MAXC];  // complex64 spectra stay complex64 in registers until they are scattered
    phi_load<NT, MAXC>(spec, src, tid, nm);
    phi_scatter<NT, MAXC>(A, spec, tid, lmax, np);
    __syncthreads();
    T stage[KP == 2 ? MAXS : 1][2];
    if (two) {
        phi_load<NT, MAXC>(spec, src + (size_t)rows * gst, tid, nm);
        if constexpr (NP > 0)
            Run::run_l(A, Tw, tid);
        else
            Run::run((double2 *)A, Pp, twp, tid, nth);
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            int col = tid + i * NT;
            col = col < cols ? col : cols - 1;
            int q = col + q0;
            q = q < 0 ? q + np : (q >= np ? q - np : q);
            const double2 v = phi_pair(ld2(A + q), k0);
            stage[KP == 2 ? i : 0][0] = (T)v.x;
            stage[KP == 2 ? i : 0][1] = (T)v.y;
        }
        __syncthreads();
        phi_scatter<NT, MAXC>(A, spec, tid, lmax, np);
        __syncthreads();
    }
    if constexpr (NP > 0)
        Run::run_l(A, Tw, tid);
    else
        Run::run((double2 *)A, Pp, twp, tid, nth);
    const int k = two ? k0 + 1 : k0;
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        const int col = tid + i * NT;
        if (col < cols) {
            int q = col + q0;
            q = q < 0 ? q + np : (q >= np ? q - np : q);
            const double2 v = phi_pair(ld2(A + q), k);
            T *o = maps + sc_map_off<T>(row, col, 2 * k0, cols, ncp);
            if (two)
                store_quad<T>(o, stage[KP == 2 ? i : 0][0], stage[KP == 2 ? i : 0][1], (T)v.x, (T)v.y);
            else
                store_pair<T>(o, v.x, v.y);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoints of the two transform stages (for the gradient with respect to the
// sky coefficients).  With <u, v> = Re sum conj(u) v on complex arrays:
//
//  phi: T_k(row, q) = sum_m G(row, m) e^{i m q h_phi} and the stored real maps
//    M_0 = Re T_0, M_1 = 0, M_{2k} = 2 Re T_k, M_{2k+1} = -2 Im T_k (wrap
//    columns are copies).  Given map gradients GM, U_k = 2 (GM_{2k} - i GM_{2k+1})
//    (U_0 = GM_0), wrap columns folded onto q mod nphi; then
//    Gadj(row, m) = sum_q e^{-i m q h_phi} U(q)  (forward FFT).
//  theta: G(r) = sum_n e^{i n r h} D_phi(m) p(n) X(n), X = FFT_{n2}(f),
//    f the parity-extended column; so Y(n) = sum_r e^{-i n r h} Gadj(r)
//    (forward FFT of the rows placed at r mod n2os), X_adj(n) =
//    conj(p(n)) D_phi(m) Y(n), f_adj = inverse FFT_{n2}(X_adj) and
//    F_adj(j) = f_adj(j) + (-1)^{m-k} f_adj(n2 - 1 - j).
template <typename T, int NT, int PT>
__global__ void __launch_bounds__(NT)
k_phi_adjoint(const T *__restrict__ gmaps, double2 *__restrict__ G, int lmax, int rows, int cols, int ncp, int W,
              FftPlan Pp, const double2 *__restrict__ twp) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int nk = gridDim.x / rows;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int row = blk / nk;
    const int k = blk - row * nk;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int np = Pp.n;
    const int q0 = -W / 2 + 1;
    double2 *A = sbuf;
    const T *src = gmaps + (size_t)row * cols * ncp;
    // columns q = 0 .. np-1 appear once at col = q - q0; the rest are wrap copies
    for (int q = tid; q < np; q += nth) {
        const T *o = src + (size_t)(q - q0) * ncp;
        A[q] = k == 0 ? make_double2((double)o[0], 0.0)
                      : make_double2(2.0 * (double)o[2 * k], -2.0 * (double)o[2 * k + 1]);
    }
    __syncthreads();
    if (tid < W - 1) {
        // the W - 1 wrap copies: cols [0, W/2 - 1) and [nphi + W/2 - 1, cols); distinct q
        const int col = tid < W / 2 - 1 ? tid : np + tid;
        const int q = col + q0;
        const int qq = q < 0 ? q + np : q - np;
        const T *o = src + (size_t)col * ncp;
        if (k == 0) {
            A[qq].x += (double)o[0];
        } else {
            A[qq].x += 2.0 * (double)o[2 * k];
            A[qq].y -= 2.0 * (double)o[2 * k + 1];
        }
    }
    __syncthreads();
    fft_lds<-1, NT, PT>(A, Pp, twp, tid, nth);
    double2 *dst = G + ((size_t)k * rows + row) * nm;
    for (int t = tid; t < nm; t += nth) {
        const int m = t - lmax;
        dst[t] = A[m < 0 ? m + np : m];
    }
}

// Two columns per workgroup, as in the forward kernel.  The forward output lies
// in the s-symmetric sequences (G(-r) = s G(r)), so the adjoint only sees the
// symmetric part of the row gradient: with A_c the gradient placed on the circle
// (zero off the kept rows), h(r) = A_1(r) + s1 A_1(-r) + i (A_2(r) - s1 A_2(-r)) is
// twice the combined symmetric input.  Its transform Y separates as in the forward
// direction, giving the combined spectrum conj(p(n)) (a Y(n) + b Y(-n)) with the
// forward kernel's a and b halved; the length-n2 inverse f keeps the parities, and
// F_adj1(j) = f(j) + s1 f(n2 - 1 - j), F_adj2(j) = -i (f(j) - s1 f(n2 - 1 - j)).
template <int NT, int PT, typename S2, typename SOS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_theta_adjoint(const double2 *__restrict__ G, double2 *__restrict__ F, int lmax, int nring, int rows, int W,
                FftPlan P2, FftPlan Pos, const double2 *__restrict__ tw2, const double2 *__restrict__ twos,
                const double2 *__restrict__ phase, const double *__restrict__ dphi) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int npair = lmax + 1;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int k = blk / npair;
    const int mi = 2 * (blk - k * npair);
    const bool two = mi + 1 < nm;
    const int m = mi - lmax;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int n2 = P2.n, nos = Pos.n;
    double2 *B = sbuf;  // length nos; the length-n2 transform runs in B[0 .. n2)
    const double s1 = ((m - k) & 1) ? -1.0 : 1.0;
    const int r0 = -W / 2 + 1;
    const int rtop = r0 + rows - 1;  // last kept row index (< nos / 2 + W)
    const double2 *gk = G + (size_t)k * rows * nm + mi;
    const double2 zero = make_double2(0.0, 0.0);
    for (int r = tid; r < nos; r += nth) {
        // kept row at circle index r (row r - r0, or a ghost row r - nos - r0), and at -r
        const int rm = r == 0 ? 0 : nos - r;
        const int ra = r <= rtop ? r - r0 : (r - nos >= r0 ? r - nos - r0 : -1);
        const int rb = rm <= rtop ? rm - r0 : (rm - nos >= r0 ? rm - nos - r0 : -1);
        double2 a1 = zero, a2 = zero, b1 = zero, b2 = zero;
        if (ra >= 0) {
            a1 = gk[(size_t)ra * nm];
            if (two) a2 = gk[(size_t)ra * nm + 1];
        }
        if (rb >= 0) {
            b1 = gk[(size_t)rb * nm];
            if (two) b2 = gk[(size_t)rb * nm + 1];
        }
        // (a1 + s1 b1) + i (a2 - s1 b2)
        const double2 u = make_double2(a1.x + s1 * b1.x, a1.y + s1 * b1.y);
        const double2 v = make_double2(a2.x - s1 * b2.x, a2.y - s1 * b2.y);
        B[r] = make_double2(u.x - v.y, u.y + v.x);
    }
    __syncthreads();
    FftRun<-1, NT, PT, SOS>::run(B, Pos, twos, tid, nth);
    // Coefficients n in [-lmax, lmax]: n >= 0 stay at n, n < 0 move from n + nos to
    // n + n2 (disjoint since nos >= n2 + lmax); the rest of [0, n2) becomes zero.
    constexpr int MAXC = (PT + 1) / 2;
    const double d1 = dphi[m < 0 ? -m : m];
    const double d2 = two ? dphi[m + 1 < 0 ? -(m + 1) : m + 1] : d1;
    const double ca = 0.25 * (d1 + d2), cb = 0.25 * s1 * (d1 - d2);
    double2 xs[MAXC];
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * nth;
        if (t < nm) {
            const int n = t - lmax;
            const double2 yp = B[n < 0 ? n + nos : n], ym = B[n > 0 ? nos - n : -n];
            const double2 y = make_double2(ca * yp.x + cb * ym.x, ca * yp.y + cb * ym.y);
            xs[i] = cmul(cconj(phase[t]), y);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXC; ++i) {
        const int t = tid + i * nth;
        if (t < nm) {
            const int n = t - lmax;
            B[n < 0 ? n + n2 : n] = xs[i];
        }
    }
    for (int t = lmax + 1 + tid; t < n2 - lmax; t += nth) B[t] = zero;
    __syncthreads();
    FftRun<1, NT, PT, S2>::run(B, P2, tw2, tid, nth);
    double2 *col = F + ((size_t)k * nm + mi) * nring;
    for (int j = tid; j < nring; j += nth) {
        const double2 a = B[j], b = B[n2 - 1 - j];
        col[j] = make_double2(a.x + s1 * b.x, a.y + s1 * b.y);
        if (two) col[nring + j] = make_double2(a.y - s1 * b.y, s1 * b.x - a.x);  // -i (a - s1 b)
    }
}

__global__ void k_widen(const float2 *__restrict__ src, double2 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = ld2(src + i);
}

}  // namespace

hipError_t sc_launch_widen(const float2 *src, double2 *dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

// Size class of a transform of length n: 0 = (256 threads, 9 points each),
// 1 = (512, 9), 2 = (1024, 9); the longest supported transform is 9216 points.
static inline int fft_class(int n) {
    return n <= SC_FFT_NT * SC_FFT_PT ? 0 : n <= SC_FFT_NT_BIG * SC_FFT_PT ? 1 : 2;
}

template <int NT, int PT, typename S2, typename SOS, typename CT>
static hipError_t theta_up_t(sc_plan *p) {
    const int nblk = (p->kmax + 1) * (p->lmax + 1);  // column pairs
    constexpr int ntw = FftRun<-1, NT, PT, S2>::ntw + FftRun<1, NT, PT, SOS>::ntw;  // zero unless both are compile-time
    // complex64 transform buffer (the kernel's choice: complex64 spectra, compile-time transforms)
    constexpr bool c64 = FftLen<S2>::value > 0 && FftLen<SOS>::value > 0 && sizeof(CT) == sizeof(float2);
    const size_t lds = (c64 ? sizeof(float2) : sizeof(double2)) * (size_t)p->n2os + sizeof(double2) * ntw;
    auto kern = k_theta_upsample<NT, PT, S2, SOS, CT, CT>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, p->stream, (const CT *)p->F, (CT *)p->G, p->lmax, p->nring,
                       p->rows, p->gst, p->W, p->p2, p->p2os, p->tw2, p->tw2os, p->phase, p->dphi);
    return hipGetLastError();
}

template <int NT, int PT, typename S2 = FftGeneric, typename SOS = FftGeneric>
static hipError_t theta_up(sc_plan *p) {
    return p->mid32 ? theta_up_t<NT, PT, S2, SOS, float2>(p) : theta_up_t<NT, PT, S2, SOS, double2>(p);
}

template <typename T, int NT, int PT, typename SP = FftGeneric>
static hipError_t phi_syn(sc_plan *p) {
    // FP32 maps with a compile-time transform: two k per workgroup (16-byte stores);
    // FP64 maps store 16 bytes per k already
    constexpr int KP = sizeof(T) == 4 && FftLen<SP>::value > 0 ? 2 : 1;
    const int nk = p->kmax + 1;
    const int nblk = (nk + KP - 1) / KP * p->rows;
    constexpr int ntw = FftRun<1, NT, PT, SP>::ntw;
    if (p->mid32) {
        const size_t lds = (FftLen<SP>::value > 0 ? sizeof(float2) : sizeof(double2)) * (size_t)p->nphi +
                           sizeof(double2) * ntw;
        auto kern = k_phi_synthesis<T, NT, PT, SP, KP, float2>;
        hipError_t e = sc_set_lds_attr((const void *)kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, p->stream, (const float2 *)p->G, (T *)p->maps, p->lmax,
                           p->rows, p->gst, p->cols, p->ncp, p->W, nk, p->pphi, p->twphi);
    } else {
        const size_t lds = sizeof(double2) * ((size_t)p->nphi + ntw);
        auto kern = k_phi_synthesis<T, NT, PT, SP, KP, double2>;
        hipError_t e = sc_set_lds_attr((const void *)kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, p->stream, (const double2 *)p->G, (T *)p->maps, p->lmax,
                           p->rows, p->gst, p->cols, p->ncp, p->W, nk, p->pphi, p->twphi);
    }
    return hipGetLastError();
}

namespace {
// The maps from their column-tiled storage into (row, column, component) order,
// one 16-byte group (G = 16 / sizeof(T) components) per thread and step.
template <typename T>
__global__ void k_maps_rowmajor(const T *__restrict__ maps, T *__restrict__ dst, int rows, int cols, int ncp) {
    constexpr int G = 16 / (int)sizeof(T);
    const int ng = ncp / G;
    const int64_t n = (int64_t)rows * cols * ng;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(i % ng);
        const int64_t rc = i / ng;
        const int r = (int)(rc / cols), c = (int)(rc - (int64_t)r * cols);
        ((uint4 *)dst)[i] = *(const uint4 *)(maps + sc_map_off<T>(r, c, G * g, cols, ncp));
    }
}
}  // namespace

template <typename T, int NT, int PT>
static hipError_t phi_adj(sc_plan *p, const void *gmaps) {
    const int nblk = (p->kmax + 1) * p->rows;
    const size_t lds = sizeof(double2) * (size_t)p->nphi;
    auto kern = k_phi_adjoint<T, NT, PT>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, p->stream, (const T *)gmaps, p->G, p->lmax,
                       p->rows, p->cols, p->ncp, p->W, p->pphi, p->twphi);
    return hipGetLastError();
}

template <int NT, int PT, typename S2 = FftGeneric, typename SOS = FftGeneric>
static hipError_t theta_adj(sc_plan *p) {
    const int nblk = (p->kmax + 1) * (p->lmax + 1);  // column pairs
    const size_t lds = sizeof(double2) * (size_t)p->n2os;
    auto kern = k_theta_adjoint<NT, PT, S2, SOS>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, p->stream, p->G, p->F, p->lmax, p->nring, p->rows, p->W,
                       p->p2, p->p2os, p->tw2, p->tw2os, p->phase, p->dphi);
    return hipGetLastError();
}

// Compile-time plans for the transform lengths of lmax 256, 512 and 1024 (radices
// chosen so each pass keeps most lanes of its waves busy, an odd radix first).
using F540 = FftSpec<540, SC_PLAN_540>;
using F1080 = FftSpec<1080, SC_PLAN_1080>;
using F2160 = FftSpec<2160, SC_PLAN_2160>;
using F4320 = FftSpec<4320, SC_PLAN_4320>;

hipError_t sc_launch_theta_upsample(sc_plan *p) {
    if (p->big) return sc_launch_theta_upsample_big(p);
    if (p->n2 == 540 && p->n2os == 1080) return theta_up<128, 9, F540, F1080>(p);
    if (p->n2 == 1080 && p->n2os == 2160) return theta_up<SC_FFT_NT, SC_FFT_PT, F1080, F2160>(p);
    if (p->n2 == 2160 && p->n2os == 4320) return theta_up<SC_FFT_NT_BIG, SC_FFT_PT, F2160, F4320>(p);
    switch (fft_class(p->n2os)) {
        case 0: return theta_up<SC_FFT_NT, SC_FFT_PT>(p);
        case 1: return theta_up<SC_FFT_NT_BIG, SC_FFT_PT>(p);
        default: return theta_up<SC_FFT_NT_HUGE, SC_FFT_PT_HUGE>(p);
    }
}

template <typename T>
static hipError_t phi_syn_any(sc_plan *p) {
    if (p->nphi == 1080) return phi_syn<T, 128, 9, F1080>(p);
    if (p->nphi == 2160) return phi_syn<T, SC_FFT_NT, SC_FFT_PT, F2160>(p);
    if (p->nphi == 4320) return phi_syn<T, SC_FFT_NT_BIG, SC_FFT_PT, F4320>(p);
    switch (fft_class(p->nphi)) {
        case 0: return phi_syn<T, SC_FFT_NT, SC_FFT_PT>(p);
        case 1: return phi_syn<T, SC_FFT_NT_BIG, SC_FFT_PT>(p);
        default: return phi_syn<T, SC_FFT_NT_HUGE, SC_FFT_PT_HUGE>(p);
    }
}

hipError_t sc_launch_phi_synthesis(sc_plan *p) {
    if (p->big) return sc_launch_phi_synthesis_big(p);
    return p->prec == SC_FP64 ? phi_syn_any<double>(p) : phi_syn_any<float>(p);
}

template <typename T>
static hipError_t phi_adj_any(sc_plan *p, const void *gmaps) {
    switch (fft_class(p->nphi)) {
        case 0: return phi_adj<T, SC_FFT_NT, SC_FFT_PT>(p, gmaps);
        case 1: return phi_adj<T, SC_FFT_NT_BIG, SC_FFT_PT>(p, gmaps);
        default: return phi_adj<T, SC_FFT_NT_HUGE, SC_FFT_PT_HUGE>(p, gmaps);
    }
}

hipError_t sc_launch_maps_rowmajor(sc_plan *p, void *dst) {
    if (p->prec == SC_FP64)
        hipLaunchKernelGGL(k_maps_rowmajor<double>, dim3(2048), dim3(256), 0, p->stream, (const double *)p->maps,
                           (double *)dst, p->rows, p->cols, p->ncp);
    else
        hipLaunchKernelGGL(k_maps_rowmajor<float>, dim3(2048), dim3(256), 0, p->stream, (const float *)p->maps,
                           (float *)dst, p->rows, p->cols, p->ncp);
    return hipGetLastError();
}

hipError_t sc_launch_phi_adjoint(sc_plan *p, const void *gmaps) {
    if (p->big) return sc_launch_phi_adjoint_big(p, gmaps);
    return p->prec == SC_FP64 ? phi_adj_any<double>(p, gmaps) : phi_adj_any<float>(p, gmaps);
}

hipError_t sc_launch_theta_adjoint(sc_plan *p) {
    if (p->big) return sc_launch_theta_adjoint_big(p);
    if (p->n2 == 540 && p->n2os == 1080) return theta_adj<128, 9, F540, F1080>(p);
    if (p->n2 == 1080 && p->n2os == 2160) return theta_adj<SC_FFT_NT, SC_FFT_PT, F1080, F2160>(p);
    if (p->n2 == 2160 && p->n2os == 4320) return theta_adj<SC_FFT_NT_BIG, SC_FFT_PT, F2160, F4320>(p);
    switch (fft_class(p->n2os)) {
        case 0: return theta_adj<SC_FFT_NT, SC_FFT_PT>(p);
        case 1: return theta_adj<SC_FFT_NT_BIG, SC_FFT_PT>(p);
        default: return theta_adj<SC_FFT_NT_HUGE, SC_FFT_PT_HUGE>(p);
    }
}
