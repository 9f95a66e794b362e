// k_gather64.hip -- FP64 interpolation + k-sum on the matrix cores (FP64 plans).
//
// The convolution at a pointing is (Galloway et al. 2022, Sec. 2.1, Eq. 8 with the
// finite-resolution maps and interpolation that follow the two-step algorithm)
//     c = sum_c basis_c(psi) X[c],   X[c] = sum_{i,j < W} w_theta(i) w_phi(j) M_c[r0 + i][q0 + j],
// basis_{2k} = cos k psi, basis_{2k+1} = sin k psi.  For the samples of one
// interpolation anchor (a work item of the binning, k_bin.hip) the inner sums are a
// matrix product over the W^2 taps t = W i + j:
//     X[c][s] = sum_t P[t][c] w_s(t),   w_s(t) = w_theta_s(i) w_phi_s(j),
// which runs here as v_mfma_f64_16x16x4_f64 (FP64 products and accumulation), so the
// result keeps the FP64 form's accuracy (1e-12 at W = 14).
//
// A persistent workgroup of 4 waves takes items from the queue.  Per item it handles
// up to S = 64 STW samples at a time (wave w owns sample tiles STW w .. STW w + STW-1);
// their 2W one-dimensional weights and e^{i psi}, e^{8 i psi} go to LDS.  The
// anchor's W x W x ncomp map block is staged in LDS one chunk of CTC component tiles
// (16 CTC components) at a time, from the last chunk down; each chunk's product
// ends in the per-sample k-sum, continued across chunks by Horner's rule.
//
// Operand layout of the 16x16x4 FP64 instruction (checked on the device): A[i][k] in
// lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), element
// i / 4.  A is the map chunk (16 components x 4 taps, row i holding component
// 4 (i % 4) + i / 4 of the tile), B the tap weights (4 taps x 16 samples), so lane
// (r = lane % 16, grp = lane / 16) ends with components 16 ct + 4 grp + v (v < 4) of
// sample r: the cos/sin pairs of orders k0 = 8 ct + 2 grp and k0 + 1.  Its part of
// the k-sum is Re[e^{2 i grp psi} sum_ct (A_ct + B_ct e^{i psi}) e^{8 i ct psi}] with
// A_ct = X[c0] - i X[c0 + 1], B_ct = X[c0 + 2] - i X[c0 + 3] (c0 = 16 ct + 4 grp),
// evaluated by Horner's rule in e^{8 i psi} from the highest tile down; the four
// lanes of a sample then add their parts.
#include "sc_common.h"

typedef double doublex4 __attribute__((ext_vector_type(4)));

namespace {

// exp(beta (sqrt(1 - z^2) - 1)) without the cancellation next to z = 0
__device__ __forceinline__ double es_weight64(double z, double beta) {
    const double z2 = z * z, q = 1.0 - z2;
    return q > 0.0 ? exp(-beta * z2 / (1.0 + sqrt(q))) : 0.0;
}

template <int W, int CTC, int STW>
struct G64 {
    static constexpr int NT = W * W;      // taps
    static constexpr int NCC = 16 * CTC;  // components per staged chunk
    static constexpr int S = 64 * STW;    // samples per pass
    static constexpr size_t lds_bytes() {
        return sizeof(double) * ((size_t)NT * NCC + 2 * W * S) + (2 * sizeof(double2) + sizeof(int)) * S;
    }
};

template <int W, int CTC, int STW>
__global__ void __launch_bounds__(256)
k_gather_mfma64(const int4 *__restrict__ items, int *__restrict__ totals, BinSorted srt,
                const double *__restrict__ maps, double *__restrict__ tod, int cols, int ncp, int ncomp, int nkc,
                double beta) {
    using G = G64<W, CTC, STW>;
    constexpr int NT = G::NT, NCC = G::NCC, S = G::S, HALF = W / 2;
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    double *P = smem_d;                         // [NT][NCC] map chunk
    double *Wt = P + NT * NCC;                  // [2W][S]: theta weights, then phi weights
    double2 *E1 = (double2 *)(Wt + 2 * W * S);  // [S] e^{i psi}
    double2 *E8 = E1 + S;                       // [S] e^{8 i psi}
    int *Idx = (int *)(E8 + S);                 // [S] sample index within the pass
    __shared__ int item_sh;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, grp = lane >> 4;
    const int nitems = totals[1];
    const int nchunks = (ncomp + NCC - 1) / NCC;
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&totals[2], 1);
        __syncthreads();
        const int it = item_sh;
        if (it >= nitems) break;
        const int4 item = items[it];
        const int row0 = item.x / nkc, col0 = item.x - (item.x / nkc) * nkc;
        for (int ch = 0; ch < item.z; ch += S) {
            const int ns = item.z - ch < S ? item.z - ch : S;
            const int pos0 = item.y + ch;
            for (int e = tid; e < 2 * W * S; e += 256) {
                const int q = e / S, sl = e - q * S;
                double w = 0.0;
                if (sl < ns) {
                    const bool th = q < W;
                    const double f = th ? srt.rec[pos0 + sl].fu : srt.rec[pos0 + sl].fv;
                    const int node = th ? q : q - W;
                    w = es_weight64((f + (double)(HALF - 1 - node)) / (double)HALF, beta);
                }
                Wt[e] = w;
            }
            for (int sl = tid; sl < S; sl += 256) {
                double ps = 0.0;
                int ix = -1;
                if (sl < ns) {
                    ps = srt.rec[pos0 + sl].psi;
                    ix = srt.rec[pos0 + sl].idx;
                }
                double sn, cs;
                sincos(ps, &sn, &cs);
                const double2 e1 = make_double2(cs, sn);
                const double2 e2 = cmul(e1, e1), e4 = cmul(e2, e2);
                E1[sl] = e1;
                E8[sl] = cmul(e4, e4);
                Idx[sl] = ix;
            }
            double2 hq[STW];
#pragma unroll
            for (int h = 0; h < STW; ++h) hq[h] = make_double2(0.0, 0.0);

            for (int cc = nchunks - 1; cc >= 0; --cc) {
                __syncthreads();  // the previous chunk's reads are done; weights and phases written
                const int cbase = cc * NCC;
                // stage the chunk: taps t of the W x W block, components cbase .. cbase + NCC - 1
                // (zero past ncomp), as 16-byte pairs (one group of the tiled maps; c is even)
#pragma unroll 4
                for (int e = tid; e < NT * (NCC / 2); e += 256) {
                    const int t = e / (NCC / 2), c2 = e - t * (NCC / 2);
                    const int c = cbase + 2 * c2;
                    const int i = t / W, j = t - (t / W) * W;
                    const double *src = maps + sc_map_off<double>(row0 + i, col0 + j, c, cols, ncp);
                    double2 v = make_double2(0.0, 0.0);
                    if (c + 1 < ncomp)
                        v = *(const double2 *)src;
                    else if (c < ncomp)
                        v.x = src[0];
                    ((double2 *)P)[e] = v;
                }
                __syncthreads();

                doublex4 acc[STW][CTC];
#pragma unroll
                for (int h = 0; h < STW; ++h)
#pragma unroll
                    for (int ct = 0; ct < CTC; ++ct) acc[h][ct] = doublex4{0.0, 0.0, 0.0, 0.0};
                // step s covers taps 4 s .. 4 s + 3; lane group grp supplies tap t = 4 s + grp,
                // (ti, tj) = (t / W, t % W) advanced by 4 per step
                int ti = 0, tj = grp;
                const double *Pa = P + grp * NCC + (4 * (r & 3) + (r >> 2));  // row r: component 4 (r % 4) + r / 4
                const double *Wth = Wt + 16 * STW * wv + r;
                const double *Wph = Wth + W * S;
#pragma unroll 2
                for (int s = 0; s < NT / 4; ++s) {
                    double a[CTC];
#pragma unroll
                    for (int ct = 0; ct < CTC; ++ct) a[ct] = Pa[4 * s * NCC + 16 * ct];
#pragma unroll
                    for (int h = 0; h < STW; ++h) {
                        const double b = Wth[ti * S + 16 * h] * Wph[tj * S + 16 * h];
#pragma unroll
                        for (int ct = 0; ct < CTC; ++ct)
                            acc[h][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ct], b, acc[h][ct], 0, 0, 0);
                    }
                    tj += 4;
                    if (tj >= W) {
                        tj -= W;
                        ++ti;
                    }
                }
                // Horner step per tile of the chunk, highest first
#pragma unroll
                for (int h = 0; h < STW; ++h) {
                    const int sl = 16 * (STW * wv + h) + r;
                    const double2 e1 = E1[sl], e8 = E8[sl];
                    double2 q = hq[h];
#pragma unroll
                    for (int ct = CTC - 1; ct >= 0; --ct) {
                        const doublex4 x = acc[h][ct];
                        // C = A + B e1 with A = x0 - i x1, B = x2 - i x3; q = q e8 + C
                        const double cx = fma(x[2], e1.x, fma(x[3], e1.y, x[0]));
                        const double cy = fma(x[2], e1.y, fma(-x[3], e1.x, -x[1]));
                        const double qx = fma(q.x, e8.x, fma(-q.y, e8.y, cx));
                        const double qy = fma(q.x, e8.y, fma(q.y, e8.x, cy));
                        q = make_double2(qx, qy);
                    }
                    hq[h] = q;
                }
            }
            // part = Re[e^{2 i grp psi} q], summed over the sample's four lane groups
#pragma unroll
            for (int h = 0; h < STW; ++h) {
                const int sl = 16 * (STW * wv + h) + r;
                const double2 e1 = E1[sl];
                const double2 e2 = cmul(e1, e1), e4 = cmul(e2, e2);
                const double2 z0 = grp == 0 ? make_double2(1.0, 0.0) : grp == 1 ? e2 : grp == 2 ? e4 : cmul(e4, e2);
                double part = z0.x * hq[h].x - z0.y * hq[h].y;
                part += __shfl_xor(part, 16);
                part += __shfl_xor(part, 32);
                if (grp == 0 && sl < ns) tod[Idx[sl]] = part;
            }
            __syncthreads();  // weights, phases and indices are rewritten by the next pass
        }
    }
}

template <int W, int CTC, int STW>
hipError_t launch64(sc_plan *p, void *tod) {
    using G = G64<W, CTC, STW>;
    static_assert(G::lds_bytes() <= 160 * 1024, "LDS");
    const size_t lds = G::lds_bytes();
    auto kern = k_gather_mfma64<W, CTC, STW>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 256, lds, p->gather_wgs_per_cu);
    const BinGeom g = sc_bin_geom(p);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, p->stream, p->bw.items, p->bw.totals, p->bw.sorted,
                       (const double *)p->maps, (double *)tod, p->cols, p->ncp, p->ncomp, g.nkc, p->beta);
    return hipGetLastError();
}

}  // namespace

// Kernel widths with an instantiation (every even width the plans accept).
bool sc_gather_mfma64_supported(int W) { return W >= 4 && W <= 16 && (W & 1) == 0; }

hipError_t sc_launch_gather_mfma64(sc_plan *p, void *tod) {
    switch (p->W) {
        case 4: return launch64<4, 4, 4>(p, tod);
        case 6: return launch64<6, 4, 4>(p, tod);
        // Two component tiles per staged chunk from W = 8 up: at lmax 512 / kmax 100 / 1e7 scan
        // samples W = 8 took 7.6 ms against 8.2 (2, 2), 8.6 (4, 2), 11.3 (8, 2), 11.5 (4, 4) and
        // 13.7 (8, 4); W = 14 took 20.9 ms against 21.7 (3, 4), 21.9 (2, 2), 22.8 (1, 4) and
        // 25.1 (3, 2) (more LDS per chunk means fewer workgroups per CU, more tiles more registers).
        case 8: return launch64<8, 2, 4>(p, tod);
        case 10: return launch64<10, 2, 4>(p, tod);
        case 12: return launch64<12, 2, 4>(p, tod);
        case 14: return launch64<14, 2, 4>(p, tod);
        case 16: return launch64<16, 2, 4>(p, tod);
        default: return hipErrorInvalidValue;
    }
}
