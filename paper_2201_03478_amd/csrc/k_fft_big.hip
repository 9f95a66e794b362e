// k_fft_big.hip -- theta upsampling and phi synthesis (and their adjoints) for
// band limits whose transforms exceed one workgroup's LDS (more than 9216 points).
//
// The stages compute what k_fft.hip computes (same grids, kernel deconvolution and
// component layout; Galloway et al. 2022, Sec. 2.1), one theta column or one
// (k, row) of the phi stage per workgroup.  A transform of length n = P N that does
// not fit is evaluated as P transforms of length N in LDS (decimation of the output
// index): for either sign DIR, with w_n = e^{DIR 2 pi i / n},
//     X[P k + s] = sum_{j < N} w_N^{j k} y_s[j],
//     y_s[j]     = w_n^{j s} sum_{q < P} x[j + N q] w_P^{q s},
// so pass s folds the input (read from global memory, where it is L2-resident),
// applies the twiddle and runs one LDS transform whose output holds every P-th
// coefficient.  Spectra that a later pass of another length must read in full go
// through a plan scratch buffer S (one padded row of 2 lmax + 1 coefficients per
// theta column).
//
// Theta columns are processed one at a time here (the small-band-limit kernels
// pair columns m and m + 1 through the parity of the extended column); with one
// column the upsampled column is simply IFFT_{n2os}(d p(n) X(n)) on the kept rows,
// X = FFT_{n2}(extended column), p(n) the half-ring phase over n2 hhat_theta(n) and
// d = 1 / hhat_phi(m).  Its exact adjoint: rows placed on the circle, forward
// transform, multiply by d conj(p(n)), inverse transform of length n2 and fold the
// extension, F_adj(j) = x(j) + s x(n2 - 1 - j), s = (-1)^{m-k}.
#include "fft_lds.h"

namespace {

constexpr int BNT = SC_FFT_NT_HUGE;  // threads per workgroup
constexpr int BPT = SC_FFT_PT_HUGE;  // points per thread (sub-transforms up to 9216 points)

__device__ __forceinline__ double2 cis_frac(int a, int n, int dir) {
    // e^{dir 2 pi i a / n}, 0 <= a < n
    double s, c;
    sincospi(2.0 * (double)dir * (double)a / (double)n, &s, &c);
    return make_double2(c, s);
}

// Pass s of a split transform of length n = P Q.n: buf <- y_s (input x(t), t < n, from
// `in`), then the LDS transform; on return buf[k] = X[P k + s].  Ends barrier-complete.
template <int DIR, typename In>
__device__ void split_pass(double2 *buf, const FftPlan &Q, const double2 *__restrict__ tw, int P, int s, int n,
                           In in, int tid) {
    const int N = Q.n;
    const double2 ws = cis_frac(s, P, DIR);  // w_P^s; w_P^{q s} by repeated products (q < P <= 16)
    for (int j = tid; j < N; j += BNT) {
        double2 acc = in(j);
        double2 wq = ws;
        for (int q = 1; q < P; ++q) {
            acc = cadd(acc, cmul(in(j + N * q), wq));
            wq = cmul(wq, ws);
        }
        if (s) acc = cmul(acc, cis_frac((int)(((long long)j * s) % n), n, DIR));
        buf[j] = acc;
    }
    __syncthreads();
    fft_lds<DIR, BNT, BPT>(buf, Q, tw, tid, BNT);
}

// Global writes of this workgroup visible to its later global reads.
__device__ __forceinline__ void wg_global_sync() {
    __threadfence();
    __syncthreads();
    __threadfence();
}

// Forward theta stage of one column (k, m): ring sums F -> rows of G.
__global__ void __launch_bounds__(BNT)
k_theta_upsample_big(const double2 *__restrict__ F, double2 *__restrict__ G, double2 *__restrict__ S, int lmax,
                     int nring, int rows, int W, int n2, int nos, int P1, FftPlan Q1, const double2 *__restrict__ tw1,
                     int P2, FftPlan Q2, const double2 *__restrict__ tw2, const double2 *__restrict__ phase,
                     const double *__restrict__ dphi, int spad) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int k = blockIdx.x / nm, mi = blockIdx.x - k * nm;
    const int m = mi - lmax;
    const int tid = threadIdx.x;
    const double s1 = ((m - k) & 1) ? -1.0 : 1.0;
    const double d = dphi[m < 0 ? -m : m];
    const double2 *col = F + ((size_t)k * nm + mi) * nring;
    double2 *spec = S + (size_t)blockIdx.x * spad;  // Z(n) at n + lmax
    const double2 zero = make_double2(0.0, 0.0);
    // extended column: x(j) = F(j), x(n2 - 1 - j) = s1 F(j)
    auto xin = [&](int t) -> double2 {
        if (t < nring) return col[t];
        const double2 v = col[n2 - 1 - t];
        return make_double2(s1 * v.x, s1 * v.y);
    };
    for (int s = 0; s < P1; ++s) {
        split_pass<-1>(sbuf, Q1, tw1, P1, s, n2, xin, tid);
        for (int kk = tid; kk < Q1.n; kk += BNT) {
            const int n = P1 * kk + s;
            const int ns = n <= n2 / 2 ? n : n - n2;
            if (ns >= -lmax && ns <= lmax) {
                const double2 z = cmul(phase[ns + lmax], sbuf[kk]);
                spec[ns + lmax] = make_double2(d * z.x, d * z.y);
            }
        }
        __syncthreads();
    }
    wg_global_sync();
    // zero-padded spectrum on the length-nos circle
    auto zin = [&](int t) -> double2 {
        if (t <= lmax) return spec[t + lmax];
        if (t >= nos - lmax) return spec[t - nos + lmax];
        return zero;
    };
    const int r0 = -W / 2 + 1, rtop = r0 + rows - 1;
    double2 *gcol = G + (size_t)k * rows * nm + mi;
    for (int s = 0; s < P2; ++s) {
        split_pass<1>(sbuf, Q2, tw2, P2, s, nos, zin, tid);
        for (int rr = tid; rr < Q2.n; rr += BNT) {
            const int r = P2 * rr + s;
            const int row = r <= rtop ? r - r0 : (r - nos >= r0 ? r - nos - r0 : -1);
            if (row >= 0) gcol[(size_t)row * nm] = sbuf[rr];
        }
        __syncthreads();
    }
}

// Map values of one k at one column, (M_{2k}, M_{2k+1}) = (2 Re T_k, -2 Im T_k) or (Re T_0, 0).
__device__ __forceinline__ double2 comp_pair(double2 v, int k) {
    return k == 0 ? make_double2(v.x, 0.0) : make_double2(2.0 * v.x, -2.0 * v.y);
}
template <typename T>
__device__ inline void put_pair(T *o, double2 v);
template <>
__device__ inline void put_pair<double>(double *o, double2 v) {
    *(double2 *)o = v;
}
template <>
__device__ inline void put_pair<float>(float *o, double2 v) {
    *(float2 *)o = make_float2((float)v.x, (float)v.y);
}

// Phi stage of one (k, row): the m-spectrum of G to the map columns (wrap copies included).
template <typename T>
__global__ void __launch_bounds__(BNT)
k_phi_synthesis_big(const double2 *__restrict__ G, T *__restrict__ maps, int lmax, int rows, int cols, int ncp, int W,
                    int nk, int nphi, int P, FftPlan Q, const double2 *__restrict__ tw) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int row = blockIdx.x / nk, k = blockIdx.x - row * nk;
    const int tid = threadIdx.x;
    const double2 *src = G + ((size_t)k * rows + row) * nm;
    const double2 zero = make_double2(0.0, 0.0);
    auto gin = [&](int t) -> double2 {
        if (t <= lmax) return src[t + lmax];
        if (t >= nphi - lmax) return src[t - nphi + lmax];
        return zero;
    };
    const int q0 = -W / 2 + 1;
    for (int s = 0; s < P; ++s) {
        split_pass<1>(sbuf, Q, tw, P, s, nphi, gin, tid);
        for (int qq = tid; qq < Q.n; qq += BNT) {
            const int q = P * qq + s;
            const double2 v = comp_pair(sbuf[qq], k);
            // column q - q0 and the wrap copies q - q0 -+ nphi inside [0, cols)
            for (int c = q - q0 - nphi; c < cols; c += nphi)
                if (c >= 0) put_pair<T>(maps + sc_map_off<T>(row, c, 2 * k, cols, ncp), v);
        }
        __syncthreads();
    }
}

// Adjoint of the phi stage for one (k, row): map gradients (wrap copies folded onto
// their column) -> forward transform -> G[k][row][m + lmax].
template <typename T>
__global__ void __launch_bounds__(BNT)
k_phi_adjoint_big(const T *__restrict__ gmaps, double2 *__restrict__ G, int lmax, int rows, int cols, int ncp, int W,
                  int nk, int nphi, int P, FftPlan Q, const double2 *__restrict__ tw) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int row = blockIdx.x / nk, k = blockIdx.x - row * nk;
    const int tid = threadIdx.x;
    const int q0 = -W / 2 + 1;
    const T *src = gmaps + (size_t)row * cols * ncp;
    auto uin = [&](int q) -> double2 {
        double2 u = make_double2(0.0, 0.0);
        for (int c = q - q0 - nphi; c < cols; c += nphi) {
            if (c < 0) continue;
            const T *o = src + (size_t)c * ncp;
            if (k == 0) {
                u.x += (double)o[0];
            } else {
                u.x += 2.0 * (double)o[2 * k];
                u.y -= 2.0 * (double)o[2 * k + 1];
            }
        }
        return u;
    };
    double2 *dst = G + ((size_t)k * rows + row) * nm;
    for (int s = 0; s < P; ++s) {
        split_pass<-1>(sbuf, Q, tw, P, s, nphi, uin, tid);
        for (int kk = tid; kk < Q.n; kk += BNT) {
            const int n = P * kk + s;
            const int ms = n <= nphi / 2 ? n : n - nphi;
            if (ms >= -lmax && ms <= lmax) dst[ms + lmax] = sbuf[kk];
        }
        __syncthreads();
    }
}

// Adjoint of the theta stage for one column: G rows -> (forward, d conj(p)) -> S ->
// inverse of length n2 -> x_adj into the column's own rows of G (read completely
// before); k_theta_fold then forms F_adj.
__global__ void __launch_bounds__(BNT)
k_theta_adjoint_big(double2 *__restrict__ G, double2 *__restrict__ S, int lmax, int rows, int W, int n2, int nos,
                    int P1, FftPlan Q1, const double2 *__restrict__ tw1, int P2, FftPlan Q2,
                    const double2 *__restrict__ tw2, const double2 *__restrict__ phase, const double *__restrict__ dphi,
                    int spad) {
    extern __shared__ double2 sbuf[];
    const int nm = 2 * lmax + 1;
    const int k = blockIdx.x / nm, mi = blockIdx.x - k * nm;
    const int m = mi - lmax;
    const int tid = threadIdx.x;
    const double d = dphi[m < 0 ? -m : m];
    double2 *gcol = G + (size_t)k * rows * nm + mi;
    double2 *spec = S + (size_t)blockIdx.x * spad;
    const double2 zero = make_double2(0.0, 0.0);
    const int r0 = -W / 2 + 1, rtop = r0 + rows - 1;
    auto ain = [&](int r) -> double2 {
        const int row = r <= rtop ? r - r0 : (r - nos >= r0 ? r - nos - r0 : -1);
        return row >= 0 ? gcol[(size_t)row * nm] : zero;
    };
    for (int s = 0; s < P2; ++s) {
        split_pass<-1>(sbuf, Q2, tw2, P2, s, nos, ain, tid);
        for (int kk = tid; kk < Q2.n; kk += BNT) {
            const int n = P2 * kk + s;
            const int ns = n <= nos / 2 ? n : n - nos;
            if (ns >= -lmax && ns <= lmax) {
                const double2 z = cmul(cconj(phase[ns + lmax]), sbuf[kk]);
                spec[ns + lmax] = make_double2(d * z.x, d * z.y);
            }
        }
        __syncthreads();
    }
    wg_global_sync();  // spectra written; every read of the column's rows is done
    auto zin = [&](int t) -> double2 {
        if (t <= lmax) return spec[t + lmax];
        if (t >= n2 - lmax) return spec[t - n2 + lmax];
        return zero;
    };
    for (int s = 0; s < P1; ++s) {
        split_pass<1>(sbuf, Q1, tw1, P1, s, n2, zin, tid);
        for (int jj = tid; jj < Q1.n; jj += BNT) gcol[(size_t)(P1 * jj + s) * nm] = sbuf[jj];
        __syncthreads();
    }
}

// F_adj(j) = x(j) + s x(n2 - 1 - j) for every column, x in rows 0 .. n2 - 1 of G.
__global__ void k_theta_fold(const double2 *__restrict__ G, double2 *__restrict__ F, int lmax, int kmax, int nring,
                             int rows) {
    const int nm = 2 * lmax + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)(kmax + 1) * nm * nring;
    if (i >= tot) return;
    const int64_t c = i / nring;
    const int j = (int)(i - c * nring);
    const int k = (int)(c / nm), mi = (int)(c - (int64_t)k * nm);
    const double s = (((mi - lmax) - k) & 1) ? -1.0 : 1.0;
    const double2 *gcol = G + (size_t)k * rows * nm + mi;
    const double2 a = gcol[(size_t)j * nm], b = gcol[(size_t)(2 * nring - 1 - j) * nm];
    F[i] = make_double2(a.x + s * b.x, a.y + s * b.y);
}

size_t big_lds(const sc_plan *p, bool theta) {
    const int n = theta ? (p->p2.n > p->p2os.n ? p->p2.n : p->p2os.n) : p->pphi.n;
    return sizeof(double2) * (size_t)n;
}

}  // namespace

hipError_t sc_launch_theta_upsample_big(sc_plan *p) {
    const size_t lds = big_lds(p, true);
    hipError_t e = sc_set_lds_attr((const void *)k_theta_upsample_big, lds);
    if (e != hipSuccess) return e;
    const int ncol = (p->kmax + 1) * (2 * p->lmax + 1);
    hipLaunchKernelGGL(k_theta_upsample_big, dim3(ncol), dim3(BNT), lds, p->stream, p->F, p->G, p->S, p->lmax,
                       p->nring, p->rows, p->W, p->n2, p->n2os, p->sp2, p->p2, p->tw2, p->spos, p->p2os, p->tw2os,
                       p->phase, p->dphi, p->spad);
    return hipGetLastError();
}

hipError_t sc_launch_phi_synthesis_big(sc_plan *p) {
    const size_t lds = big_lds(p, false);
    const int nk = p->kmax + 1;
    const unsigned nblk = (unsigned)(nk * p->rows);
    hipError_t e;
    if (p->prec == SC_FP64) {
        e = sc_set_lds_attr((const void *)k_phi_synthesis_big<double>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_synthesis_big<double>, dim3(nblk), dim3(BNT), lds, p->stream, p->G,
                           (double *)p->maps, p->lmax, p->rows, p->cols, p->ncp, p->W, nk, p->nphi, p->spphi, p->pphi,
                           p->twphi);
    } else {
        e = sc_set_lds_attr((const void *)k_phi_synthesis_big<float>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_synthesis_big<float>, dim3(nblk), dim3(BNT), lds, p->stream, p->G,
                           (float *)p->maps, p->lmax, p->rows, p->cols, p->ncp, p->W, nk, p->nphi, p->spphi, p->pphi,
                           p->twphi);
    }
    return hipGetLastError();
}

hipError_t sc_launch_phi_adjoint_big(sc_plan *p, const void *gmaps) {
    const size_t lds = big_lds(p, false);
    const int nk = p->kmax + 1;
    const unsigned nblk = (unsigned)(nk * p->rows);
    hipError_t e;
    if (p->prec == SC_FP64) {
        e = sc_set_lds_attr((const void *)k_phi_adjoint_big<double>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_adjoint_big<double>, dim3(nblk), dim3(BNT), lds, p->stream, (const double *)gmaps,
                           p->G, p->lmax, p->rows, p->cols, p->ncp, p->W, nk, p->nphi, p->spphi, p->pphi, p->twphi);
    } else {
        e = sc_set_lds_attr((const void *)k_phi_adjoint_big<float>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_adjoint_big<float>, dim3(nblk), dim3(BNT), lds, p->stream, (const float *)gmaps,
                           p->G, p->lmax, p->rows, p->cols, p->ncp, p->W, nk, p->nphi, p->spphi, p->pphi, p->twphi);
    }
    return hipGetLastError();
}

hipError_t sc_launch_theta_adjoint_big(sc_plan *p) {
    const size_t lds = big_lds(p, true);
    hipError_t e = sc_set_lds_attr((const void *)k_theta_adjoint_big, lds);
    if (e != hipSuccess) return e;
    const int ncol = (p->kmax + 1) * (2 * p->lmax + 1);
    hipLaunchKernelGGL(k_theta_adjoint_big, dim3(ncol), dim3(BNT), lds, p->stream, p->G, p->S, p->lmax, p->rows, p->W,
                       p->n2, p->n2os, p->sp2, p->p2, p->tw2, p->spos, p->p2os, p->tw2os, p->phase, p->dphi, p->spad);
    const int64_t tot = (int64_t)ncol * p->nring;
    hipLaunchKernelGGL(k_theta_fold, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, p->stream, p->G, p->F, p->lmax,
                       p->kmax, p->nring, p->rows);
    return hipGetLastError();
}
