// k_gather.hip -- interpolation of the component maps and the per-sample k-sum.
//
// For a pointing (theta, phi, psi) the convolution is (Galloway et al. 2022,
// Sec. 2.1, Eq. 8 with the finite-resolution maps and interpolation described
// after the two-step algorithm)
//     c = sum_{i,j < W} w_theta(i) w_phi(j) sum_c basis_c(psi) M_c[r0 + i][q0 + j],
//     basis = (1, 0, cos psi, sin psi, cos 2 psi, sin 2 psi, ...)
//     (basis_{2k} = cos k psi, basis_{2k+1} = sin k psi; the stored sin 0 psi map is zero),
// with exponential-of-semicircle weights w(z) = exp(beta (sqrt(1 - z^2) - 1)),
// z = (x - x_node) / (W/2) in grid units.  The grid indices and the fractional
// offsets are formed in FP64 (a float phi near 2 pi would misplace the stencil
// by up to 2.4e-7 rad); psi is reduced in FP64 before its multiples are taken.
//
// v1 layout: one wave per sample, lanes over components.
#include "sc_common.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {
// Work-queue runs: with more than GATHER_RUN_DIV items per workgroup the persistent
// gather takes up to 32 consecutive items per queue atomic; GATHER_SLIDE enables the
// reuse of the staged block between consecutive items of a run (split form).
constexpr int GATHER_RUN_DIV = 64;
constexpr bool GATHER_SLIDE = true;
}  // namespace

namespace {

int ct_class(int ncomp);

// exp(beta (sqrt(1 - z^2) - 1)) as exp(-beta z^2 / (1 + sqrt(1 - z^2))): no cancellation next to
// z = 0, where the weights are largest
template <typename T>
__device__ __forceinline__ T es_weight(T z, T beta) {
    const T z2 = z * z, q = (T)1 - z2;
    return q > (T)0 ? exp(-beta * z2 / ((T)1 + sqrt(q))) : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gather_v1(const double *__restrict__ ptg, int64_t n, const T *__restrict__ maps, T *__restrict__ tod, int cols,
            int ncp, int ncomp, int W, double beta, double inv_hth, double inv_hph, int n2os, int nphi) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int half = W / 2;
    const double two_pi = 6.283185307179586477;
    for (int64_t s = wave; s < n; s += nwaves) {
        const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
        double u = th * inv_hth;
        u = fmin(fmax(u, 0.0), 0.5 * (double)n2os);
        const int r0 = (int)floor(u) - half + 1;
        double v = (ph - two_pi * floor(ph / two_pi)) * inv_hph;
        if (!(v < (double)nphi)) v = 0.0;  // 2 pi rounding, NaN
        if (v < 0.0) v = 0.0;
        const int q0 = (int)floor(v) - half + 1;
        T w = (T)0;
        if (lane < W)
            w = es_weight<T>((T)((u - (double)(r0 + lane)) / half), (T)beta);
        else if (lane < 2 * W)
            w = es_weight<T>((T)((v - (double)(q0 + lane - W)) / half), (T)beta);

        T acc[4] = {(T)0, (T)0, (T)0, (T)0};
        const int row0 = r0 + half - 1, col0 = q0 + half - 1;
        for (int i = 0; i < W; ++i) {
            const T wi = __shfl(w, i);
            for (int j = 0; j < W; ++j) {
                const T wij = wi * __shfl(w, W + j);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = lane + 64 * t;
                    if (c < ncomp) acc[t] += wij * maps[sc_map_off<T>(row0 + i, col0 + j, c, cols, ncp)];
                }
            }
        }
        double psr = ps - two_pi * floor(ps / two_pi);
        T part = (T)0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = lane + 64 * t;
            if (c < ncomp) {
                double sn, cs;
                sincos((double)(c >> 1) * psr, &sn, &cs);
                part += (T)((c & 1) ? sn : cs) * acc[t];
            }
        }
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
        if (lane == 0) tod[s] = part;
    }
}

// ---------------------------------------------------------------------------
// Binned gather (W = 8).  A persistent workgroup takes work items from a queue;
// an item is up to BIN_CHUNK samples that share the stencil anchor (row0, col0)
// (see k_bin.hip).  The 8 x 8 x ncomp map block of the anchor is staged in LDS
// once; the samples are processed 64 at a time as a register-blocked product
//     X[s][c] = sum_{t < 64} w_s(t) P[t][c]      (w_s(t) = w_theta(i) w_phi(j))
// with each lane holding 4 samples x CPT consecutive components, followed by
// the k-sum sum_c basis_c(psi_s) X[s][c] and a reduction over the 16 lanes that
// hold the components of a sample.
//
// cos k psi / sin k psi in FP64: one sincos per sample gives e^{i psi}; a table
// of e^{i k0(g) psi} at the first order k0(g) of each of the 16 component groups
// is built by powers and a 16-step product chain (error ~16 ulp), and each lane
// rotates from its group's entry by e^{i psi} (at most CPT/2 + 1 steps).
__device__ __forceinline__ double2 cpowi(double2 z, int n) {
    double2 r = make_double2(1.0, 0.0);
    while (n) {
        if (n & 1) r = cmul(r, z);
        z = cmul(z, z);
        n >>= 1;
    }
    return r;
}

template <typename T, int CPT>
__global__ void __launch_bounds__(256)
k_gather_binned(const int4 *__restrict__ items, int *__restrict__ totals, BinSorted srt,
                const T *__restrict__ maps, T *__restrict__ tod, int cols, int ncp, int ncomp, int nkc,
                double beta) {
    constexpr int NC = 16 * CPT;  // staged components (zero-padded)
    extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte operands
    T *Psh = (T *)smem_d;         // [64 taps][NC]
    T *Wsh = Psh + 64 * NC;       // [64 taps][64 samples]; reused for Eg after the product
    double2 *Eg = (double2 *)Wsh; // [64 samples][16 groups] e^{i k0(g) psi}
    T *W1 = Wsh + 64 * 64;        // [16][64 samples]: 8 theta then 8 phi weights
    double2 *E1 = (double2 *)(W1 + 64 * 16);  // [64] (cos psi, sin psi)
    int *Idx = (int *)(E1 + 64);              // [64]
    __shared__ int item_sh;

    const int tid = threadIdx.x;
    const int sg = tid >> 4, cg = tid & 15;
    const int nitems = totals[1];
    const T tbeta = (T)beta;
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&totals[2], 1);
        __syncthreads();
        const int it = item_sh;
        if (it >= nitems) break;
        const int4 item = items[it];
        const int row0 = item.x / nkc, col0 = item.x - (item.x / nkc) * nkc;
        for (int e = tid; e < 64 * NC; e += 256) {
            const int t = e / NC, c = e - t * NC;
            T v = (T)0;
            if (c < ncp) v = maps[sc_map_off<T>(row0 + (t >> 3), col0 + (t & 7), c, cols, ncp)];
            Psh[e] = v;
        }
        for (int ch = 0; ch < item.z; ch += 64) {
            const int ns = item.z - ch < 64 ? item.z - ch : 64;
            const int pos0 = item.y + ch;
            for (int e = tid; e < 64 * 16; e += 256) {
                const int q = e >> 6, sl = e & 63;
                T w = (T)0;
                if (sl < ns) {
                    const T f = (q < 8) ? (T)srt.rec[pos0 + sl].fu : (T)srt.rec[pos0 + sl].fv;
                    const T z = (f + (T)(3 - (q & 7))) * (T)0.25;  // (x - node) / (W/2)
                    w = es_weight<T>(z, tbeta);
                }
                W1[e] = w;
            }
            if (tid < 64) {
                double ps = 0.0;
                int ix = -1;
                if (tid < ns) {
                    ps = srt.rec[pos0 + tid].psi;
                    ix = srt.rec[pos0 + tid].idx;
                }
                double sn, cs;
                sincos(ps, &sn, &cs);
                E1[tid] = make_double2(cs, sn);
                Idx[tid] = ix;
            }
            __syncthreads();
            for (int e = tid; e < 64 * 64; e += 256) {
                const int t = e >> 6, sl = e & 63;
                Wsh[e] = W1[(t >> 3) * 64 + sl] * W1[(8 + (t & 7)) * 64 + sl];
            }
            __syncthreads();

            T acc[4][CPT];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < CPT; ++c) acc[q][c] = (T)0;
#pragma unroll 4
            for (int t = 0; t < 64; ++t) {
                const T *wr = Wsh + t * 64 + 4 * sg;
                const T w0 = wr[0], w1 = wr[1], w2 = wr[2], w3 = wr[3];
                const T *pr = Psh + t * NC + cg * CPT;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const T pv = pr[c];
                    acc[0][c] = fma(w0, pv, acc[0][c]);
                    acc[1][c] = fma(w1, pv, acc[1][c]);
                    acc[2][c] = fma(w2, pv, acc[2][c]);
                    acc[3][c] = fma(w3, pv, acc[3][c]);
                }
            }
            __syncthreads();  // Wsh is dead: build the group phase table in its place
            {
                const int sl = tid >> 2, q = tid & 3;  // 4 lanes per sample, 4 groups each
                const double2 e1 = E1[sl];
                int kc = ((4 * q) * CPT) >> 1;
                double2 z = cpowi(e1, kc);
#pragma unroll
                for (int g = 4 * q; g < 4 * q + 4; ++g) {
                    const int k0 = (g * CPT) >> 1;
                    if (k0 > kc) {
                        z = cmul(z, cpowi(e1, k0 - kc));
                        kc = k0;
                    }
                    Eg[sl * 16 + g] = z;
                }
            }
            __syncthreads();

            const int c0 = cg * CPT;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int sl = 4 * sg + q;
                const double2 e1 = E1[sl];
                double2 z = Eg[sl * 16 + cg];
                int k = c0 >> 1;
                T part = (T)0;
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    const int c = c0 + j;
                    if (c < ncomp) {
                        if ((c >> 1) > k) {
                            z = cmul(z, e1);
                            ++k;
                        }
                        part = fma((T)((c & 1) ? z.y : z.x), acc[q][j], part);
                    }
                }
                part += __shfl_xor(part, 8);
                part += __shfl_xor(part, 4);
                part += __shfl_xor(part, 2);
                part += __shfl_xor(part, 1);
                if (cg == 0 && sl < ns) tod[Idx[sl]] = part;
            }
            __syncthreads();
        }
    }
}

template <typename T, int CPT>
hipError_t launch_binned(sc_plan *p, void *tod) {
    constexpr int NC = 16 * CPT;
    static_assert(64 * 64 * sizeof(T) >= 64 * 16 * sizeof(double2), "group table must fit the weight area");
    const size_t lds = sizeof(T) * (64 * NC + 64 * 64 + 64 * 16) + 64 * (sizeof(double2) + sizeof(int));
    auto kern = k_gather_binned<T, CPT>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 256, lds, p->gather_wgs_per_cu);
    const BinGeom g = sc_bin_geom(p);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, p->stream, p->bw.items, p->bw.totals,
                       p->bw.sorted, (const T *)p->maps, (T *)tod, p->cols, p->ncp, p->ncomp, g.nkc, p->beta);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_binned_t(sc_plan *p, void *tod) {
    const int cpt = (p->ncomp + 15) / 16;
    if (cpt <= 1) return launch_binned<T, 1>(p, tod);
    if (cpt <= 2) return launch_binned<T, 2>(p, tod);
    if (cpt <= 3) return launch_binned<T, 3>(p, tod);
    if (cpt <= 5) return launch_binned<T, 5>(p, tod);
    if (cpt <= 9) return launch_binned<T, 9>(p, tod);
    if (cpt <= 13) return launch_binned<T, 13>(p, tod);
    return launch_binned<T, 16>(p, tod);
}


// ---------------------------------------------------------------------------
// Binned gather on the matrix cores (FP32 maps).  Same work items and weights as
// k_gather_binned; per chunk of up to 128 samples the product
//     Y[c][s] = sum_{t < 64} P[t][c] w_s(t)     (16 CT comps x 128 samples x 64 taps)
// runs as v_mfma_f32_16x16x4_f32 (FP32 products, FP32 accumulation) with the
// map block P as the A operand and the tap weights w_s(t) = w_theta w_phi as B
// (formed on the fly from the two 8-tap factors); a workgroup of NWV = 4 or 8
// waves takes 128 samples, wave w owning 8/NWV 16-sample tiles and all component
// tiles (8 waves hold half the accumulators each and double the waves per CU).  Operand layout of
// the 16x16x4 instruction: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in lane j + 16(i/4), register i%4.  Lane (r = lane%16, grp = lane/16)
// therefore holds components c = 16 ct + 4 grp + v (v < 4) of ONE sample
// (16 (TPW w + h) + r): the cos/sin pairs of orders k0 = 8 ct + 2 grp and k0 + 1,
// reached from e^{i 2 grp psi} by FP64 rotations with e^{i psi} and
// e^{i 8 psi}; the sum over the lane's components is completed
// across the four lanes of the sample.
// Map rows in LDS are padded to a stride of NC + 16 floats when the tile count
// is even, and the weight rows to 144 floats, so the four lane groups of an
// operand read fall in distinct bank quarters.
constexpr int GCH = 128;       // samples per chunk
constexpr int GW1 = GCH + 16;  // weight row stride (floats)

__host__ __device__ constexpr size_t mfma_lds_bytes(int CT) {
    return sizeof(float) * (64 * (16 * (size_t)CT + 16) + 16 * GW1) + GCH * (sizeof(double2) + sizeof(int));
}

// The k-sum of one chunk: lane (r, grp) of wave w holds, for each of its TPW
// sample tiles h, components 16 ct + 4 grp + v of sample s0 + 16 h (s0 =
// 16 TPW w + r); it forms sum_c basis_c(psi) X[c] over them, the four lanes of
// the sample add their parts, and the sum (times oscale) is the sample's value.
// With k0 = 8 ct + 2 grp the lane's four components are the pairs of k0 and
// k0 + 1, so its part is Re[e^{2 i grp psi} sum_ct (A_ct + B_ct e^{i psi}) w^ct]
// with A_ct = X[c0] - i X[c0 + 1], B_ct = X[c0 + 2] - i X[c0 + 3] and w = e^{8 i psi},
// evaluated by Horner's rule in w (FP64).  Component tiles other than the last are
// full (the padded count is the next multiple of 16); the last one's components
// past ncomp are left out.
template <int CT, int TPW>
__device__ __forceinline__ void ksum_store(const GatherDet &D, const floatx4 (&acc)[TPW][CT], const double2 *E,
                                           const int *Idx, int s0, int grp, int ns, float oscale) {
#pragma unroll
    for (int h = 0; h < TPW; ++h) {
        const int sl = s0 + 16 * h;
        const double2 e1 = E[sl];  // (cos psi, sin psi) of the sample
        const double2 e2 = cmul(e1, e1), e4 = cmul(e2, e2);
        const double2 e8 = cmul(e4, e4);
        const double2 z0 = grp == 0 ? make_double2(1.0, 0.0) : grp == 1 ? e2 : grp == 2 ? e4 : cmul(e4, e2);
        double2 q = make_double2(0.0, 0.0);
#pragma unroll
        for (int ct = CT - 1; ct >= 0; --ct) {
            const int c0 = 16 * ct + 4 * grp;
            const floatx4 x = acc[h][ct];
            double ax = (double)x[0], ay = -(double)x[1], bx = (double)x[2], by = -(double)x[3];
            if (ct == CT - 1) {
                if (c0 >= D.ncomp) ax = ay = 0.0;
                if (c0 + 2 >= D.ncomp) bx = by = 0.0;
            }
            // C = A + B e1;  q = q w + C
            const double cx = fma(bx, e1.x, fma(-by, e1.y, ax));
            const double cy = fma(bx, e1.y, fma(by, e1.x, ay));
            const double qx = fma(q.x, e8.x, fma(-q.y, e8.y, cx));
            const double qy = fma(q.x, e8.y, fma(q.y, e8.x, cy));
            q = make_double2(qx, qy);
        }
        double part = z0.x * q.x - z0.y * q.y;
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (grp == 0 && sl < ns) D.tod[Idx[sl]] = (float)part * oscale;
    }
}

// One work item: stage the anchor's map block, then contract its samples GCH at a
// time.  CT is the item's exact component-tile count (a compile-time constant,
// so the product loop has no per-tile branches and its LDS loads run ahead of
// the matrix instructions).
template <int CT, int NWV>
__device__ __forceinline__ void gather_mfma_item(const GatherDet &D, const int4 item, double *smem_d) {
    constexpr int NT = 64 * NWV;    // threads
    constexpr int TPW = 8 / NWV;    // 16-sample tiles per wave
    constexpr int NC = 16 * CT;                   // == D.ncp for the FP32 forms
    constexpr int NCS = NC + ((CT & 1) ? 0 : 16); // LDS row stride
    float *Psh = (float *)smem_d;                 // [64 taps][NCS]
    float *W1 = Psh + 64 * NCS;                   // [16][GW1]: theta (0..7) and phi (8..15) factors
    double2 *E = (double2 *)(W1 + 16 * GW1);      // [GCH] (cos psi, sin psi)
    int *Idx = (int *)(E + GCH);                  // [GCH]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, grp = lane >> 4;
    const int row0 = item.x / D.nkc, col0 = item.x - (item.x / D.nkc) * D.nkc;
    // Sample records of the next chunk are loaded into registers one chunk
    // ahead (thread t stages the weights of sample t % GCH; threads < GCH also
    // carry psi and the output index), so their latency overlaps the products.
    const int sw = tid & (GCH - 1);
    double pf_u = 0.0, pf_v = 0.0, pf_psi = 0.0;
    int pf_idx = -1;
    {
        const int ns0 = item.z < GCH ? item.z : GCH;
        if (sw < ns0) {
            pf_u = D.srt.rec[item.y + sw].fu;
            pf_v = D.srt.rec[item.y + sw].fv;
        }
        if (tid < ns0) {
            pf_psi = D.srt.rec[item.y + tid].psi;
            pf_idx = D.srt.rec[item.y + tid].idx;
        }
    }
    {
        // tap t = 8 i + j is map row row0 + i, column col0 + j: NC / 4 groups of four components
        const int n4 = NC / 4, ntile = sc_map_ntile(D.cols);
        for (int t = wv; t < 64; t += NWV) {
            float4 *d4 = (float4 *)(Psh + t * NCS);
            for (int q = lane; q < n4; q += 64)
                d4[q] = *(const float4 *)(D.maps + sc_tile_off(row0 + (t >> 3), col0 + (t & 7), q, ntile, n4));
        }
    }
    for (int ch = 0; ch < item.z; ch += GCH) {
        const int ns = item.z - ch < GCH ? item.z - ch : GCH;
        {
            const float fu = (float)pf_u, fv = (float)pf_v;
            const float nbl = -D.beta * 1.44269504088896341f;  // -beta log2(e)
#pragma unroll
            for (int i = 0; i < 16 * GCH / NT; ++i) {
                const int q = (tid >> 7) + (NT / GCH) * i;  // NT threads cover NT / GCH weight rows per step
                float w = 0.f;
                if (sw < ns) w = es_weight_f32(((q < 8 ? fu : fv) + (float)(3 - (q & 7))) * 0.25f, nbl);
                W1[q * GW1 + sw] = w;
            }
        }
        if (tid < GCH) {
            double sn, cs;  // once per sample (the k-sum's four lanes of a sample share it)
            sincos(tid < ns ? pf_psi : 0.0, &sn, &cs);
            E[tid] = make_double2(cs, sn);
            Idx[tid] = tid < ns ? pf_idx : -1;
        }
        __syncthreads();
        {
            const int nxt = ch + GCH;
            const int nns = item.z - nxt < GCH ? item.z - nxt : GCH;  // <= 0 past the last chunk
            if (sw < nns) {
                pf_u = D.srt.rec[item.y + nxt + sw].fu;
                pf_v = D.srt.rec[item.y + nxt + sw].fv;
            }
            if (tid < nns) {
                pf_psi = D.srt.rec[item.y + nxt + tid].psi;
                pf_idx = D.srt.rec[item.y + nxt + tid].idx;
            }
        }

        floatx4 acc[TPW][CT];
#pragma unroll
        for (int h = 0; h < TPW; ++h)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[h][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int s0 = 16 * TPW * wv + r;
        const float *pa = Psh + grp * NCS + r;  // A[i = comp r][k = tap grp] of component tile 0
        // Software pipeline: the operands of tap group ks + 1 (map values and the
        // two weight factors) are read from LDS before the matrix instructions of
        // group ks are issued, and multiplied only after them.
        float a[CT], ft[TPW], fp[TPW];
        {
            const float *wt = W1 + (grp >> 3) * GW1, *wp = W1 + (8 + (grp & 7)) * GW1;
#pragma unroll
            for (int h = 0; h < TPW; ++h) {
                ft[h] = wt[s0 + 16 * h];
                fp[h] = wp[s0 + 16 * h];
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) a[ct] = pa[16 * ct];
        }
#pragma unroll 2
        for (int ks = 0; ks < 16; ++ks) {
            float bw[TPW];
#pragma unroll
            for (int h = 0; h < TPW; ++h) bw[h] = ft[h] * fp[h];
            float an[CT];
            const int ksn = ks + 1 < 16 ? ks + 1 : ks;  // last group: harmless re-read
            {
                const int tap = 4 * ksn + grp;
                const float *wt = W1 + (tap >> 3) * GW1, *wp = W1 + (8 + (tap & 7)) * GW1;
#pragma unroll
                for (int h = 0; h < TPW; ++h) {
                    ft[h] = wt[s0 + 16 * h];
                    fp[h] = wp[s0 + 16 * h];
                }
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) an[ct] = pa[ksn * 4 * NCS + 16 * ct];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ct], bw[h], acc[h][ct], 0, 0, 0);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) a[ct] = an[ct];
        }

        ksum_store<CT, TPW>(D, acc, E, Idx, s0, grp, ns, 1.f);
        __syncthreads();  // W1, E, Idx are rewritten by the next chunk
    }
}

// ---------------------------------------------------------------------------
// Split products on the FP16/FP8 matrix cores, to FP32 accuracy.  A map value
// x (FP32, 24 significant bits) is written exactly as x = a1 + a2 + a3 with
// a1 = fp16(x), a2 = fp16(x - a1) (round to nearest; 11 + 11 bits) and the
// remainder a3 = x - a1 - a2, which has at most 2 significant bits and is held
// exactly in FP8 (e4m3).  A tap weight w is written as b1 + b2 (two FP16 parts,
// |w - b1 - b2| <= 2^-22 w) and as fp8(w).  The product is
//     x w ~ a1 b1 + a1 b2 + a2 b1 + a2 b2 + a3 fp8(w)
// (the omitted terms are below 2^-26 |x w|): four v_mfma_f32_16x16x32_f16 and
// one v_mfma_f32_16x16x32_fp8_fp8, FP32 accumulation, i.e. 9/32 of the matrix
// time of the FP32 form.  The map values carry all 24 bits because their
// rounding errors are amplified by the cancellation in the k-sum; the weight's
// 2^-22 is not (a weight multiplies every component of its tap alike).
// Ranges are handled by exact power-of-two scalings: the map block of an item
// by 2^(15 - e) with 2^e above its largest magnitude (a workgroup max taken
// while the block is staged), the weights by 2^14 (FP16 parts) and the
// remainders a3 by 2^14 (FP8); the k-sum undoes them.  Values far below the
// block maximum lose relative, not absolute, precision in the subnormal
// ranges: an absolute error below 2^-37 of the block maximum.
//
// Operand layout of the 16x16x32 instructions: A[i][k] in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; D as for the
// FP32 form.  Taps are grouped in two halves of 32 (map rows 0-3 and 4-7);
// within a half, lane group g holds map row 4 half + g and element q the map
// column q, for A (component r of tile ct) and B (sample r of tile h) alike.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

constexpr float SPLIT_WSCALE = 16384.f;  // 2^14
constexpr float SPLIT_RSCALE = 16384.f;  // 2^14

__host__ __device__ constexpr size_t split_lds_bytes(int CT) {
    return 2 * (2 * (size_t)CT * 64 * sizeof(half8)) + 2 * (size_t)CT * 64 * sizeof(long) + sizeof(float) * 16 * GW1 +
           GCH * (sizeof(double2) + sizeof(int));
}

// An empty use of a register value (keeps it allocated up to this point).
template <typename V>
__device__ __forceinline__ void keep_live(const V &v) {
    asm volatile("" ::"v"(v));
}

// The value as computed (rounded to FP32 and held in a register): the compiler
// cannot fold the operation that produced it into a later conversion.
__device__ __forceinline__ float as_is(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

// eight floats to eight FP8 (e4m3) bytes, element q in byte q
__device__ __forceinline__ long pack_fp8x8(const float (&f)[8]) {
    int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(f[0], f[1], 0, false);
    w0 = __builtin_amdgcn_cvt_pk_fp8_f32(f[2], f[3], w0, true);
    int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(f[4], f[5], 0, false);
    w1 = __builtin_amdgcn_cvt_pk_fp8_f32(f[6], f[7], w1, true);
    return (long)(((unsigned long)(unsigned)w1 << 32) | (unsigned)w0);
}

// Block reuse between consecutive items of one workgroup (LDS).  Work items come
// in anchor order, and the next anchor is usually the next column of the same map
// row, so its 8 x 8 block shares seven columns with the staged one.  The staged
// block keeps its columns in slots: map column c sits in element c mod 8 of every
// operand vector (the phi weight rows of W1 are permuted to match), so moving one
// column on replaces one slot.  Each item's block is split with the scale of its
// own maximum, as a freshly staged block is (the per-slot maxima are kept), so the
// products and the result do not depend on which items a workgroup took before.
struct SlideLds {
    int key;              // anchor of the staged block (-2: none)
    int e;                // its scale exponent (block maximum < 2^e)
    unsigned smax8[8];    // maximum |value| of each slot's column (float bits)
    unsigned wmax[8][8];  // per-wave slot maxima while a block is staged
};

template <int CT, int NWV, bool SLIDE = false>
__device__ __forceinline__ void gather_split_item(const GatherDet &D, const int4 item, double *smem_d, unsigned *smax,
                                                  SlideLds *sl = nullptr, bool reuse = false) {
    constexpr int NT = 64 * NWV;
    constexpr int TPW = 8 / NWV;
    constexpr int NC = 16 * CT;
    constexpr int NC4 = NC / 4;
    constexpr int NU = 8 * NC4;                // staging units: (map row, 4 components) x 8 columns
    constexpr int UPT = (NU + NT - 1) / NT;
    half8 *Ahi = (half8 *)smem_d;              // [2 tap halves][CT][64 lanes]: a1
    half8 *Alo = Ahi + 2 * CT * 64;            // a2
    long *Arm = (long *)(Alo + 2 * CT * 64);   // a3 (FP8 x 8)
    float *W1 = (float *)(Arm + 2 * CT * 64);  // [16][GW1]: theta (0..7) and phi (8..15) factors
    double2 *E = (double2 *)(W1 + 16 * GW1);   // [GCH] (cos psi, sin psi)
    int *Idx = (int *)(E + GCH);               // [GCH]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, grp = lane >> 4;
    const int row0 = item.x / D.nkc, col0 = item.x - (item.x / D.nkc) * D.nkc;
    // column col0 + jj of a (row, four-component group): the group's run in col0's tile,
    // then (col0 mod 8 + jj >= 8) the same group in the next tile, 32 (NC4 - 1) floats on
    const int ntile = sc_map_ntile(D.cols), cm8 = col0 & 7;
    auto col_at = [&](const float *b0, int jj) -> const floatx4 * {
        return (const floatx4 *)(b0 + 4 * jj + (cm8 + jj >= 8 ? 32 * (NC4 - 1) : 0));
    };
    const int sw = tid & (GCH - 1);
    double pf_u = 0.0, pf_v = 0.0, pf_psi = 0.0;
    int pf_idx = -1;
    {
        const int ns0 = item.z < GCH ? item.z : GCH;
        if (sw < ns0) {
            pf_u = D.srt.rec[item.y + sw].fu;
            pf_v = D.srt.rec[item.y + sw].fv;
        }
        if (tid < ns0) {
            pf_psi = D.srt.rec[item.y + tid].psi;
            pf_idx = D.srt.rec[item.y + tid].idx;
        }
    }
    float oscale;
    int e = 0;
    bool restage = true;
    // slot of map column col0 + j (j < 8): element j, or (col0 + j) mod 8 with block reuse
    const bool track = SLIDE && reuse;  // slot order and block reuse (uniform)
    const int c7 = track ? (col0 & 7) : 0;
    if (track) {
        const int skey = sl->key;
        if (item.x == skey) {
            restage = false;  // the same anchor (a large one split into several items)
            e = sl->e;
        } else if (item.x == skey + 1 && col0 != 0) {
            // one column on: stage column col0 + 7 into slot (col0 + 7) mod 8, unless the
            // block's scale changes
            const int snew = (col0 + 7) & 7;
            constexpr int NU1 = 8 * NC4;  // (map row, 4 components) units of one column
            constexpr int UP1 = (NU1 + NT - 1) / NT;
            floatx4 nv[UP1];
            float m = 0.f;
#pragma unroll
            for (int k = 0; k < UP1; ++k) {
                const int u = tid + k * NT;
                nv[k] = floatx4{0.f, 0.f, 0.f, 0.f};
                if (u < NU1) {
                    const int i = u / NC4, c4 = u - i * NC4;
                    nv[k] = *col_at(D.maps + sc_tile_off(row0 + i, col0, c4, ntile, NC4), 7);
                }
                m = fmaxf(m, fmaxf(fmaxf(fabsf(nv[k][0]), fabsf(nv[k][1])), fmaxf(fabsf(nv[k][2]), fabsf(nv[k][3]))));
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
            if (lane == 0) atomicMax(smax, __float_as_uint(m));
            __syncthreads();
            const unsigned mnew = *smax;
            unsigned mb = mnew;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j != snew) mb = max(mb, sl->smax8[j]);
            int eb;
            (void)frexpf(__uint_as_float(mb), &eb);
            if (eb == sl->e) {
                restage = false;
                e = eb;
                const float ms = ldexpf(1.f, 15 - e);
#pragma unroll
                for (int k = 0; k < UP1; ++k) {
                    const int u = tid + k * NT;
                    if (u < NU1) {
                        const int i = u / NC4, c4 = u - i * NC4;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int c = 4 * c4 + q;
                            const float x = as_is(nv[k][q] * ms);  // the same split as a staged block's
                            const _Float16 h1 = (_Float16)x;
                            const float r1 = as_is(x - (float)h1);
                            const _Float16 h2 = (_Float16)r1;
                            const float rm = (r1 - (float)h2) * SPLIT_RSCALE;
                            const int o = ((i >> 2) * CT + (c >> 4)) * 64 + (i & 3) * 16 + (c & 15);
                            ((_Float16 *)(Ahi + o))[snew] = h1;
                            ((_Float16 *)(Alo + o))[snew] = h2;
                            ((unsigned char *)(Arm + o))[snew] =
                                (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(rm, 0.f, 0, false) & 0xff);
                        }
                    }
                }
                if (tid == 0) sl->smax8[snew] = mnew;  // no thread reads this slot's entry again before a barrier
            }
        }
    }
    if (restage) {
        floatx4 v[UPT][8];
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int u = tid + k * NT;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[k][j] = floatx4{0.f, 0.f, 0.f, 0.f};
            if (u < NU) {
                const int i = u / NC4, c4 = u - i * NC4;
                const float *b0 = D.maps + sc_tile_off(row0 + i, col0, c4, ntile, NC4);
                // slot j holds map column col0 + ((j - col0) mod 8)
#pragma unroll
                for (int j = 0; j < 8; ++j) v[k][j] = *col_at(b0, (j - c7) & 7);
            }
            if (!track) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    m = fmaxf(m, fmaxf(fmaxf(fabsf(v[k][j][0]), fabsf(v[k][j][1])),
                                       fmaxf(fabsf(v[k][j][2]), fabsf(v[k][j][3]))));
            }
        }
        if (track) {
            // per-slot maxima (a wave reduction per slot), kept for the next items
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float mj = 0.f;
#pragma unroll
                for (int k = 0; k < UPT; ++k)
                    mj = fmaxf(mj, fmaxf(fmaxf(fabsf(v[k][j][0]), fabsf(v[k][j][1])),
                                         fmaxf(fabsf(v[k][j][2]), fabsf(v[k][j][3]))));
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) mj = fmaxf(mj, __shfl_xor(mj, off));
                if (lane == 0) sl->wmax[wv][j] = __float_as_uint(mj);
            }
            __syncthreads();
            unsigned mb = 0u;
#pragma unroll
            for (int w = 0; w < NWV; ++w)
#pragma unroll
                for (int j = 0; j < 8; ++j) mb = max(mb, sl->wmax[w][j]);
            if (tid < 8) {
                unsigned mj = 0u;
#pragma unroll
                for (int w = 0; w < NWV; ++w) mj = max(mj, sl->wmax[w][tid]);
                sl->smax8[tid] = mj;
            }
            (void)frexpf(__uint_as_float(mb), &e);  // block maximum < 2^e
        } else {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
            if (lane == 0) atomicMax(smax, __float_as_uint(m));  // non-negative floats order as their bits
            __syncthreads();
            (void)frexpf(__uint_as_float(*smax), &e);  // block maximum < 2^e
        }
        const float ms = ldexpf(1.f, 15 - e);
        oscale = ldexpf(1.f, e - 15) * (1.f / SPLIT_WSCALE);
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int u = tid + k * NT;
            if (u < NU) {
                const int i = u / NC4, c4 = u - i * NC4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 4 * c4 + q;
                    half8 hi, lo;
                    float rm[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float x = as_is(v[k][j][q] * ms);  // exact (power of two)
                        hi[j] = (_Float16)x;
                        const float r1 = as_is(x - (float)hi[j]);  // exact
                        lo[j] = (_Float16)r1;
                        rm[j] = (r1 - (float)lo[j]) * SPLIT_RSCALE;  // exact; <= 2 significant bits
                    }
                    const int o = ((i >> 2) * CT + (c >> 4)) * 64 + (i & 3) * 16 + (c & 15);
                    Ahi[o] = hi;
                    Alo[o] = lo;
                    Arm[o] = pack_fp8x8(rm);
                }
            }
        }
    }
    if (track) {
        if (!restage) oscale = ldexpf(1.f, e - 15) * (1.f / SPLIT_WSCALE);
        if (tid == 0) {  // read by the next item after the barriers below
            sl->key = item.x;
            sl->e = e;
        }
    }
    for (int ch = 0; ch < item.z; ch += GCH) {
        const int ns = item.z - ch < GCH ? item.z - ch : GCH;
        {
            const float fu = (float)pf_u, fv = (float)pf_v;
            const float nbl = -D.beta * 1.44269504088896341f;  // -beta log2(e)
            // col0 mod 8 (recomputed from the item, not held across the staging)
            const int cslot = track ? ((item.x - (item.x / D.nkc) * D.nkc) & 7) : 0;
#pragma unroll
            for (int i = 0; i < 16 * GCH / NT; ++i) {
                const int q = (tid >> 7) + (NT / GCH) * i;
                float w = 0.f;
                if (sw < ns) w = es_weight_f32(((q < 8 ? fu : fv) + (float)(3 - (q & 7))) * 0.25f, nbl);
                W1[(track && q >= 8 ? 8 + ((q + cslot) & 7) : q) * GW1 + sw] = w;  // phi factor of column col0 + j: slot row
            }
        }
        if (tid < GCH) {
            double sn, cs;  // once per sample (the k-sum's four lanes of a sample share it)
            sincos(tid < ns ? pf_psi : 0.0, &sn, &cs);
            E[tid] = make_double2(cs, sn);
            Idx[tid] = tid < ns ? pf_idx : -1;
        }
        __syncthreads();
        {
            const int nxt = ch + GCH;
            const int nns = item.z - nxt < GCH ? item.z - nxt : GCH;
            if (sw < nns) {
                pf_u = D.srt.rec[item.y + nxt + sw].fu;
                pf_v = D.srt.rec[item.y + nxt + sw].fv;
            }
            if (tid < nns) {
                pf_psi = D.srt.rec[item.y + nxt + tid].psi;
                pf_idx = D.srt.rec[item.y + nxt + tid].idx;
            }
        }

        floatx4 acc[TPW][CT];
#pragma unroll
        for (int h = 0; h < TPW; ++h)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[h][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int s0 = 16 * TPW * wv + r;
        float wph[TPW][8];
#pragma unroll
        for (int h = 0; h < TPW; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j) wph[h][j] = W1[(8 + j) * GW1 + s0 + 16 * h] * SPLIT_WSCALE;
        // Software pipeline over the 2 CT (tap half, component tile) steps: the map
        // operands of step q + 1 are read from LDS before the products of step q.
        const half8 *ph = Ahi + lane, *pl = Alo + lane;  // step q = kh CT + ct at 64 q
        const long *pr = Arm + lane;
        half8 ah = ph[0], al = pl[0];
        long ar = pr[0];
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            half8 bh[TPW], bl[TPW];
            long b8[TPW];
#pragma unroll
            for (int h = 0; h < TPW; ++h) {
                const float wt = W1[(4 * kh + grp) * GW1 + s0 + 16 * h];
                float w8[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    // one rounding of the product, and both parts split from that value
                    // (fusing the product into either conversion would pair the two
                    // parts with differently rounded products)
                    const float x = as_is(wt * wph[h][j]);
                    bh[h][j] = (_Float16)x;
                    bl[h][j] = (_Float16)(x - (float)bh[h][j]);
                    w8[j] = x * (1.f / SPLIT_RSCALE);
                }
                b8[h] = pack_fp8x8(w8);
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int q = kh * CT + ct;
                const int qn = q + 1 < 2 * CT ? q + 1 : q;
                const half8 ahn = ph[64 * qn], aln = pl[64 * qn];
                const long arn = pr[64 * qn];
                __builtin_amdgcn_sched_barrier(0);
                // smallest terms first
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ar, b8[h], acc[h][ct], 0, 0, 0);
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bl[h], acc[h][ct], 0, 0, 0);
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[h], acc[h][ct], 0, 0, 0);
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[h], acc[h][ct], 0, 0, 0);
#pragma unroll
                for (int h = 0; h < TPW; ++h)
                    acc[h][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[h], acc[h][ct], 0, 0, 0);
                // The operands stay live past their products (the barrier keeps the
                // products above these uses), so that no product's destination is
                // allocated over its own A or B registers.
                __builtin_amdgcn_sched_barrier(0);
                keep_live(ah);
                keep_live(al);
                keep_live(ar);
#pragma unroll
                for (int h = 0; h < TPW; ++h) {
                    keep_live(bh[h]);
                    keep_live(bl[h]);
                    keep_live(b8[h]);
                }
                ah = ahn;
                al = aln;
                ar = arn;
            }
        }
        ksum_store<CT, TPW>(D, acc, E, Idx, s0, grp, ns, oscale);
        __syncthreads();  // W1, E, Idx are rewritten by the next chunk
    }
}

template <int CT, int NWV, int MM, bool SLIDE = false>
__device__ __forceinline__ void gather_item(const GatherDet &D, const int4 item, double *smem_d, unsigned *smax,
                                            SlideLds *sl = nullptr, bool reuse = false) {
    if constexpr (MM == SC_MMA_SPLIT16)
        gather_split_item<CT, NWV, SLIDE>(D, item, smem_d, smax, sl, reuse);
    else
        gather_mfma_item<CT, NWV>(D, item, smem_d);
}

__host__ __device__ constexpr size_t gather_lds_bytes(int MM, int CT) {
    return MM == SC_MMA_SPLIT16 ? split_lds_bytes(CT) : mfma_lds_bytes(CT);
}

template <int CT, int NWV, int MM>
__global__ void __launch_bounds__(64 * NWV, NWV / 2)
k_gather_mfma(GatherDet D, int *__restrict__ cursor) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte operands
    __shared__ int item_sh;
    __shared__ unsigned smax;  // block / new-column maximum of the split form, cleared before every item
    const int nitems = D.totals[1];
    // Up to 8 component tiles (where the registers fit beside the accumulators), the
    // split form takes its items in runs of consecutive ones when there are many
    // short items (over ~64 per workgroup): one queue atomic per run instead of per
    // item (the single counter is contended otherwise), and since consecutive items
    // are mostly neighbouring anchors the run reuses the staged block.
    constexpr bool SL = GATHER_SLIDE && MM == SC_MMA_SPLIT16 && CT <= 8;
    if constexpr (SL) {
        __shared__ SlideLds sl;  // the staged block
        int run = nitems / (GATHER_RUN_DIV * (int)gridDim.x);
        run = run < 1 ? 1 : (run > 32 ? 32 : run);
        const bool reuse = run > 1;
        if (threadIdx.x == 0) {
            item_sh = atomicAdd(cursor, run);
            smax = 0u;
            sl.key = -2;
            sl.e = 0;
        }
        __syncthreads();
        int it = __builtin_amdgcn_readfirstlane(item_sh);
        while (it < nitems) {
            int nxt = 0;
            if (threadIdx.x == 0) nxt = atomicAdd(cursor, run);  // the next run, taken while this one runs
            const int iend = __builtin_amdgcn_readfirstlane(it + run < nitems ? it + run : nitems);
            for (int j = it; j < iend; ++j) {
                gather_item<CT, NWV, MM, true>(D, D.items[j], smem_d, &smax, &sl, reuse);  // ends with a barrier
                if (threadIdx.x == 0) smax = 0u;
                __syncthreads();
            }
            if (threadIdx.x == 0) item_sh = nxt;
            __syncthreads();
            it = __builtin_amdgcn_readfirstlane(item_sh);
        }
    } else {
        if (threadIdx.x == 0) {
            item_sh = atomicAdd(cursor, 1);
            smax = 0u;
        }
        __syncthreads();
        int it = item_sh;
        while (it < nitems) {
            int nxt = 0;
            if (threadIdx.x == 0) nxt = atomicAdd(cursor, 1);  // the next item, taken while this one runs
            gather_item<CT, NWV, MM>(D, D.items[it], smem_d, &smax);  // ends with a barrier
            if (threadIdx.x == 0) {
                item_sh = nxt;
                smax = 0u;
            }
            __syncthreads();
            it = item_sh;
        }
    }
}

// Item routine for a runtime tile count ct in [1, CTMAX]: one instantiation per count.
template <int CT, int CTMAX, int NWV, int MM>
__device__ __forceinline__ void gather_item_ct(const GatherDet &D, const int4 item, double *smem_d, unsigned *smax,
                                               int ct) {
    if (ct == CT || CT == CTMAX) {
        gather_item<CT, NWV, MM>(D, item, smem_d, smax);
        return;
    }
    if constexpr (CT < CTMAX) gather_item_ct<CT + 1, CTMAX, NWV, MM>(D, item, smem_d, smax, ct);
}

// All detectors of a batch in one persistent launch: one queue over the items
// of every detector (detector d's items follow detector d-1's); each item runs
// with its detector's component-tile count (<= CTMAX).
template <int CTMAX, int NWV, int MM>
__global__ void __launch_bounds__(64 * NWV, NWV / 2)
k_gather_batch(const GatherDet *__restrict__ dets, int ndet, int *__restrict__ cursor) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte operands
    __shared__ int start[SC_MAX_DET + 1];
    __shared__ int item_sh;
    __shared__ unsigned smax;
    if (threadIdx.x == 0) {
        smax = 0u;
        int s = 0;
        for (int d = 0; d < ndet; ++d) {
            start[d] = s;
            s += dets[d].totals[1];
        }
        start[ndet] = s;
    }
    __syncthreads();
    const int total = start[ndet];
    if (threadIdx.x == 0) item_sh = atomicAdd(cursor, 1);
    __syncthreads();
    int it = item_sh;
    while (it < total) {
        int nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(cursor, 1);  // the next item, taken while this one runs
        int d = 0;
        while (d + 1 < ndet && it >= start[d + 1]) ++d;
        const GatherDet D = dets[d];
        gather_item_ct<1, CTMAX, NWV, MM>(D, D.items[it - start[d]], smem_d, &smax, (D.ncomp + 15) / 16);  // ends with a barrier
        if (threadIdx.x == 0) {
            item_sh = nxt;
            smax = 0u;
        }
        __syncthreads();
        it = item_sh;
    }
}

// Component tiles as instantiated: 1, 2, 3, 5, 9, 13, 16.
int ct_class(int ncomp) {
    const int ct = (ncomp + 15) / 16;
    if (ct <= 3) return ct < 1 ? 1 : ct;
    if (ct <= 5) return 5;
    if (ct <= 9) return 9;
    if (ct <= 13) return 13;
    return 16;
}

template <int CT, int NWV, int MM>
hipError_t launch_mfma(sc_plan *p, void *tod) {
    const size_t lds = gather_lds_bytes(MM, CT);
    auto kern = k_gather_mfma<CT, NWV, MM>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 64 * NWV, lds, p->gather_wgs_per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NWV), lds, p->stream, sc_gather_det(p, tod), p->bw.totals + 2);
    return hipGetLastError();
}

template <int CT, int NWV, int MM>
hipError_t launch_mfma_ct(sc_plan *p, void *tod, int ct) {
    if (ct == CT || CT == 16) return launch_mfma<CT, NWV, MM>(p, tod);
    if constexpr (CT < 16) return launch_mfma_ct<CT + 1, NWV, MM>(p, tod, ct);
    return hipErrorInvalidValue;
}

template <int NWV, int MM>
hipError_t launch_mfma_w(sc_plan *p, void *tod) {
    return launch_mfma_ct<1, NWV, MM>(p, tod, (p->ncomp + 15) / 16);  // exact tile count, 1 .. 16
}

// The split form always runs 4-wave workgroups (its 8-wave build, limited to 128
// registers per lane, spills heavily and is not used).
hipError_t launch_mfma_any(sc_plan *p, void *tod) {
    if (p->gather_mma == SC_MMA_SPLIT16) return launch_mfma_w<4, SC_MMA_SPLIT16>(p, tod);
    return p->gather_waves == 8 ? launch_mfma_w<8, SC_MMA_FP32>(p, tod) : launch_mfma_w<4, SC_MMA_FP32>(p, tod);
}
}  // namespace

// FP32 maps: W = 8.  FP64 maps: every even width (k_gather64.hip stages the block
// in component chunks); the VALU form above is kept for W = 8 as a comparison
// (env SC_GATHER_PATH=valu).
bool sc_gather_binned_supported(const sc_plan *p) {
    if (p->prec == SC_FP64) return sc_gather_mfma64_supported(p->W) && p->ncomp <= 256;
    return p->W == 8 && p->ncomp <= 256;
}

hipError_t sc_launch_gather_binned(sc_plan *p, void *tod) {
    if (p->prec == SC_FP64)
        return p->gather_valu && p->W == 8 && p->ncomp <= 208 ? launch_binned_t<double>(p, tod)
                                                             : sc_launch_gather_mfma64(p, tod);
    if (p->gather_valu) return launch_binned_t<float>(p, tod);
    return launch_mfma_any(p, tod);
}

GatherDet sc_gather_det(const sc_plan *p, void *tod) {
    GatherDet D;
    D.items = p->bw.items;
    D.totals = p->bw.totals;
    D.srt = p->bw.sorted;
    D.maps = (const float *)p->maps;
    D.tod = (float *)tod;
    D.cols = p->cols;
    D.ncp = p->ncp;
    D.ncomp = p->ncomp;
    D.nkc = sc_bin_geom(p).nkc;
    D.beta = (float)p->beta;
    D.ct = ct_class(p->ncomp);
    return D;
}

template <int CTMAX, int NWV, int MM>
static hipError_t gather_batch(const GatherDet *dets_dev, int ndet, int *cursor, int wgs_per_cu, hipStream_t stream) {
    const size_t lds = gather_lds_bytes(MM, CTMAX);
    auto kern = k_gather_batch<CTMAX, NWV, MM>;
    hipError_t e = sc_set_lds_attr((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int grid = sc_persistent_grid((const void *)kern, 64 * NWV, lds, wgs_per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NWV), lds, stream, dets_dev, ndet, cursor);
    return hipGetLastError();
}

template <int NWV, int MM>
static hipError_t gather_batch_w(const GatherDet *dets_dev, int ndet, int max_ct, int *cursor, int wgs_per_cu,
                                 hipStream_t stream) {
    if (max_ct <= 2) return gather_batch<2, NWV, MM>(dets_dev, ndet, cursor, wgs_per_cu, stream);
    if (max_ct <= 5) return gather_batch<5, NWV, MM>(dets_dev, ndet, cursor, wgs_per_cu, stream);
    if (max_ct <= 13) return gather_batch<13, NWV, MM>(dets_dev, ndet, cursor, wgs_per_cu, stream);
    return gather_batch<16, NWV, MM>(dets_dev, ndet, cursor, wgs_per_cu, stream);
}

// One persistent launch over the binned items of several FP32 plans; max_ct is
// the largest component-tile count among them, waves the workgroup shape of the
// FP32 form (4 or 8; the split form runs 4), mma the product form.
hipError_t sc_launch_gather_batch(const GatherDet *dets_dev, int ndet, int max_ct, int *cursor, int wgs_per_cu,
                                  int waves, int mma, hipStream_t stream) {
    if (mma == SC_MMA_SPLIT16) return gather_batch_w<4, SC_MMA_SPLIT16>(dets_dev, ndet, max_ct, cursor, wgs_per_cu, stream);
    return waves == 8 ? gather_batch_w<8, SC_MMA_FP32>(dets_dev, ndet, max_ct, cursor, wgs_per_cu, stream)
                      : gather_batch_w<4, SC_MMA_FP32>(dets_dev, ndet, max_ct, cursor, wgs_per_cu, stream);
}

hipError_t sc_launch_gather(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    const double two_pi = 6.283185307179586477;
    const double inv_hth = (double)p->n2os / two_pi, inv_hph = (double)p->nphi / two_pi;
    int64_t nblk = (n + 3) / 4;
    if (nblk > 65536) nblk = 65536;
    if (p->prec == SC_FP64)
        hipLaunchKernelGGL(k_gather_v1<double>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const double *)p->maps, (double *)tod, p->cols, p->ncp, p->ncomp, p->W, p->beta,
                           inv_hth, inv_hph, p->n2os, p->nphi);
    else
        hipLaunchKernelGGL(k_gather_v1<float>, dim3((unsigned)nblk), dim3(256), 0, p->stream, ptg, n,
                           (const float *)p->maps, (float *)tod, p->cols, p->ncp, p->ncomp, p->W, p->beta,
                           inv_hth, inv_hph, p->n2os, p->nphi);
    return hipGetLastError();
}
