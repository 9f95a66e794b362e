// k_dipole.hip -- orbital dipole and quadrupole seen through the full beam.
//
// The kinematic signal of the satellite's motion is, to second order in
// beta = v / c, D(n) = T0 [beta.n + q (beta.n)^2] (Galloway et al. 2022,
// Sec. 3.3, Eqs. 14-16).  It is not fixed on the sky, so it is not part of the
// precomputed maps; instead its convolution with the beam reduces to the
// beam's first and second moments in the beam frame,
//     S_i = int n_i b(n) dOmega,   S_ij = int n_i n_j b(n) dOmega   (Eqs. 17-19),
// and for a pointing R = R_z(phi) R_y(theta) R_z(psi) (beam frame -> sky) with
// u = R^T beta,
//     D~ = T0 [u.S + q u^T S2 u].
// The moments depend only on the l <= 2 beam coefficients.  With the real
// field b(n) = sum_lk b_lk Y_lk (Condon-Shortley phase, b_{l,-k} =
// (-1)^k conj(b_lk)) and the l = 1, 2 harmonics written out in x, y, z:
//     S_x = -sqrt(8 pi / 3) Re b_11,   S_y = sqrt(8 pi / 3) Im b_11,   S_z = sqrt(4 pi / 3) b_10,
//     S_zz = sqrt(4 pi) b_00 / 3 + sqrt(16 pi / 5) b_20 / 3,
//     S_xz = -sqrt(8 pi / 15) Re b_21,   S_yz = sqrt(8 pi / 15) Im b_21,
//     S_xx - S_yy = sqrt(32 pi / 15) Re b_22,   S_xy = -sqrt(32 pi / 15) Im b_22 / 2,
//     S_xx + S_yy = sqrt(4 pi) b_00 - S_zz.
// One thread per sample (FP64): the velocity is stored once per pointing period
// (samples_per_period consecutive samples share it), the rotation is applied
// as three plane rotations, and the result is one FP64 value.  The workgroup's
// first thread forms the nine moments from the coefficients into LDS.
#include "sc_common.h"

namespace {

// alm-layout index of (l, k), k >= 0: k (2 lmax + 1 - k) / 2 + l
__device__ __forceinline__ double2 coef(const double2 *blm, int lmax, int kmax, int l, int k) {
    if (l > lmax || k > kmax || k > l) return make_double2(0.0, 0.0);
    return blm[(size_t)k * (2 * lmax + 1 - k) / 2 + l];
}

__global__ void __launch_bounds__(256)
k_dipole_response(const double2 *__restrict__ blm, int lmax, int kmax, const double *__restrict__ ptg, int64_t n,
                  const double *__restrict__ beta, int64_t spp, double T0, double q, double *__restrict__ out) {
    __shared__ double Sm[9];  // S_x, S_y, S_z, S_xx, S_yy, S_zz, S_xy, S_xz, S_yz
    if (threadIdx.x == 0) {
        const double pi = 3.14159265358979323846;
        const double b00 = coef(blm, lmax, kmax, 0, 0).x, b10 = coef(blm, lmax, kmax, 1, 0).x;
        const double b20 = coef(blm, lmax, kmax, 2, 0).x;
        const double2 b11 = coef(blm, lmax, kmax, 1, 1), b21 = coef(blm, lmax, kmax, 2, 1);
        const double2 b22 = coef(blm, lmax, kmax, 2, 2);
        const double c1 = sqrt(8.0 * pi / 3.0), c2 = sqrt(8.0 * pi / 15.0), c3 = sqrt(32.0 * pi / 15.0);
        const double i1 = sqrt(4.0 * pi) * b00;  // int b dOmega
        const double szz = i1 / 3.0 + sqrt(16.0 * pi / 5.0) * b20 / 3.0;
        const double dxy = c3 * b22.x;             // S_xx - S_yy
        Sm[0] = -c1 * b11.x;
        Sm[1] = c1 * b11.y;
        Sm[2] = sqrt(4.0 * pi / 3.0) * b10;
        Sm[3] = 0.5 * (i1 - szz + dxy);
        Sm[4] = 0.5 * (i1 - szz - dxy);
        Sm[5] = szz;
        Sm[6] = -0.5 * c3 * b22.y;
        Sm[7] = -c2 * b21.x;
        Sm[8] = c2 * b21.y;
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
    const double *bv = beta + 3 * (s / spp);
    double st, ct, sp, cp, ss, cs;
    sincos(th, &st, &ct);
    sincos(ph, &sp, &cp);
    sincos(ps, &ss, &cs);
    // u = R^T beta = R_z(-psi) R_y(-theta) R_z(-phi) beta
    const double v1x = cp * bv[0] + sp * bv[1], v1y = -sp * bv[0] + cp * bv[1], v1z = bv[2];
    const double v2x = ct * v1x - st * v1z, v2z = st * v1x + ct * v1z;
    const double ux = cs * v2x + ss * v1y, uy = -ss * v2x + cs * v1y, uz = v2z;
    const double lin = ux * Sm[0] + uy * Sm[1] + uz * Sm[2];
    const double quad = ux * ux * Sm[3] + uy * uy * Sm[4] + uz * uz * Sm[5] +
                        2.0 * (ux * uy * Sm[6] + ux * uz * Sm[7] + uy * uz * Sm[8]);
    out[s] = T0 * (lin + q * quad);
}

}  // namespace

hipError_t sc_launch_dipole(const double *blm, int lmax, int kmax, const double *ptg, int64_t n, const double *beta,
                            int64_t spp, double T0, double q, double *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_dipole_response, dim3((unsigned)nb), dim3(256), 0, stream, (const double2 *)blm, lmax,
                       kmax, ptg, n, beta, spp, T0, q, out);
    return hipGetLastError();
}
