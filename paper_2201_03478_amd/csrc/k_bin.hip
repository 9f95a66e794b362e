// k_bin.hip -- pointing preprocessing: bin samples by interpolation anchor.
//
// The interpolation stencil of a pointing starts at the grid node
// (row0, col0) = (floor(theta / h_theta), floor(phi / h_phi)) in map storage
// coordinates; every sample with the same anchor reads the same W x W x ncomp
// block of the component maps.  A counting sort groups the samples by anchor
// so that the gather can stage one block in LDS and reuse it for all of them:
//
//   k_bin_keys     anchor key and rank within the key per sample (counts
//                  aggregated per workgroup in LDS, one global atomic per key)
//   k_scan_*       exclusive scan of (samples, work items) per key
//   k_bin_scatter  sample records in key order: fractional offsets and psi
//                  (FP64) and the original index, 32 bytes each
//   k_bin_items    work items (key, first sorted sample, count <= the plan's bin chunk)
//
// Integer index arithmetic is exact; the fractional offsets u - floor(u) are
// kept in FP64 (the FP32 gather rounds them when it forms its weights).
#include "sc_common.h"

namespace {

__global__ void k_fill_int(int *a, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__device__ __forceinline__ void anchor_of(const double *ptg, int64_t s, const BinGeom &g, int &row0, int &col0,
                                          double &fu, double &fv, double &psi) {
    const double two_pi = 6.283185307179586477;
    const double th = ptg[3 * s], ph = ptg[3 * s + 1], ps = ptg[3 * s + 2];
    double u = th * g.inv_hth;
    u = fmin(fmax(u, 0.0), 0.5 * (double)g.n2os);  // also maps NaN to 0
    double v = (ph - two_pi * floor(ph / two_pi)) * g.inv_hph;
    if (!(v < (double)g.nphi) || v < 0.0) v = 0.0;
    const double flu = floor(u), flv = floor(v);
    row0 = (int)flu;
    col0 = (int)flv;
    fu = u - flu;
    fv = v - flv;
    psi = ps - two_pi * floor(ps / two_pi);
    if (!(psi >= 0.0 && psi < two_pi)) psi = 0.0;
}

// Anchor key and rank within the key.  A scan crosses about one anchor cell per
// sample but retraces nearly the same cells on consecutive spin circles, so a
// workgroup's span of consecutive samples hits each of its keys several times.
// The workgroup counts its keys in an LDS hash table (local ranks from LDS
// atomics), then reserves one global range per distinct key (one global atomic
// per key instead of per sample): rank = global base + local rank.  Keys that find
// no free slot within the probe limit take a global rank directly.  Ranges of
// different workgroups, and direct ranks, are disjoint by construction.
constexpr int KEYS_NT = 1024;        // threads per workgroup
constexpr int KEYS_SPT = 16;         // samples per thread (a span of 16384 samples)
constexpr int KEYS_HT = 4096;        // hash slots
constexpr int KEYS_PROBE = 64;       // linear-probe limit
constexpr int KEYS_EMPTY = -1;

__global__ void __launch_bounds__(KEYS_NT) k_bin_keys(const double *__restrict__ ptg, int64_t n, BinGeom g,
                                                      int *__restrict__ key, int *__restrict__ rank,
                                                      int *__restrict__ count) {
    __shared__ int hkey[KEYS_HT];
    __shared__ int hcnt[KEYS_HT];  // local count, then the key's global base
    const int tid = threadIdx.x;
    for (int i = tid; i < KEYS_HT; i += KEYS_NT) {
        hkey[i] = KEYS_EMPTY;
        hcnt[i] = 0;
    }
    __syncthreads();
    const int64_t s0 = (int64_t)blockIdx.x * (KEYS_NT * KEYS_SPT);
    int kk[KEYS_SPT], slot[KEYS_SPT], lr[KEYS_SPT];
#pragma unroll
    for (int i = 0; i < KEYS_SPT; ++i) {  // all keys first: the pointing loads overlap
        const int64_t s = s0 + tid + (int64_t)i * KEYS_NT;
        kk[i] = -1;
        if (s < n) {
            int r0, c0;
            double fu, fv, psi;
            anchor_of(ptg, s, g, r0, c0, fu, fv, psi);
            kk[i] = r0 * g.nkc + c0;
            key[s] = kk[i];
        }
    }
#pragma unroll
    for (int i = 0; i < KEYS_SPT; ++i) {
        const int k = kk[i];
        slot[i] = -1;
        lr[i] = 0;
        if (k >= 0) {
            int h = (int)(((unsigned)k * 2654435761u) >> 20) & (KEYS_HT - 1);
            for (int q = 0; q < KEYS_PROBE; ++q) {
                int cur = hkey[h];
                if (cur == KEYS_EMPTY) cur = atomicCAS(&hkey[h], KEYS_EMPTY, k);
                if (cur == KEYS_EMPTY || cur == k) {
                    slot[i] = h;
                    lr[i] = atomicAdd(&hcnt[h], 1);
                    break;
                }
                h = (h + 1) & (KEYS_HT - 1);
            }
            if (slot[i] < 0) lr[i] = atomicAdd(&count[k], 1);  // table full along the probe path
        }
    }
    __syncthreads();
    for (int i = tid; i < KEYS_HT; i += KEYS_NT) {
        const int k = hkey[i];
        if (k != KEYS_EMPTY) hcnt[i] = atomicAdd(&count[k], hcnt[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KEYS_SPT; ++i) {
        const int64_t s = s0 + tid + (int64_t)i * KEYS_NT;
        if (s < n) rank[s] = slot[i] >= 0 ? hcnt[slot[i]] + lr[i] : lr[i];
    }
}

// --- exclusive scan of int2 (x: samples per key, y: items per key) ------------
constexpr int SCAN_NT = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_BLOCK = SCAN_NT * SCAN_PER;

__device__ __forceinline__ int2 key_pair(const int *count, int64_t i, int64_t nkeys, int chunk) {
    if (i >= nkeys) return make_int2(0, 0);
    const int c = count[i];
    return make_int2(c, (c + chunk - 1) / chunk);
}

// block-wide exclusive scan of one int2 per thread; returns the block total
__device__ int2 block_scan(int2 v, int2 *sh, int &excl_x, int &excl_y) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_NT; off <<= 1) {
        int2 t = tid >= off ? sh[tid - off] : make_int2(0, 0);
        __syncthreads();
        sh[tid] = make_int2(sh[tid].x + t.x, sh[tid].y + t.y);
        __syncthreads();
    }
    const int2 incl = sh[tid];
    excl_x = incl.x - v.x;
    excl_y = incl.y - v.y;
    const int2 tot = sh[SCAN_NT - 1];
    __syncthreads();
    return tot;
}

__global__ void __launch_bounds__(SCAN_NT) k_scan_reduce(const int *__restrict__ count, int64_t nkeys,
                                                         int2 *__restrict__ sums, int chunk) {
    __shared__ int2 sh[SCAN_NT];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER;
    int2 acc = make_int2(0, 0);
    for (int q = 0; q < SCAN_PER; ++q) {
        const int2 v = key_pair(count, base + q, nkeys, chunk);
        acc.x += v.x;
        acc.y += v.y;
    }
    int ex, ey;
    const int2 tot = block_scan(acc, sh, ex, ey);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the per-block sums; writes totals
__global__ void __launch_bounds__(SCAN_NT) k_scan_sums(int2 *__restrict__ sums, int nblk, int *__restrict__ totals) {
    __shared__ int2 sh[SCAN_NT];
    int2 carry = make_int2(0, 0);
    for (int base = 0; base < nblk; base += SCAN_NT) {
        const int i = base + threadIdx.x;
        const int2 v = i < nblk ? sums[i] : make_int2(0, 0);
        int ex, ey;
        const int2 tot = block_scan(v, sh, ex, ey);
        if (i < nblk) sums[i] = make_int2(carry.x + ex, carry.y + ey);
        carry.x += tot.x;
        carry.y += tot.y;
    }
    if (threadIdx.x == 0) {
        totals[0] = carry.x;  // samples
        totals[1] = carry.y;  // work items
        totals[2] = 0;        // work-queue cursor of the gather
    }
}

__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const int *__restrict__ count, int64_t nkeys,
                                                        const int2 *__restrict__ sums, int2 *__restrict__ offs,
                                                        int chunk) {
    __shared__ int2 sh[SCAN_NT];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER;
    int2 v[SCAN_PER];
    int2 acc = make_int2(0, 0);
    for (int q = 0; q < SCAN_PER; ++q) {
        v[q] = key_pair(count, base + q, nkeys, chunk);
        acc.x += v[q].x;
        acc.y += v[q].y;
    }
    int ex, ey;
    block_scan(acc, sh, ex, ey);
    const int2 bo = sums[blockIdx.x];
    int2 run = make_int2(bo.x + ex, bo.y + ey);
    for (int q = 0; q < SCAN_PER; ++q) {
        if (base + q < nkeys) offs[base + q] = run;
        run.x += v[q].x;
        run.y += v[q].y;
    }
}

// Sample records in anchor order.  Lane pairs write the two 16-byte halves of one
// record in the same instruction (one 32-byte run per sample, not four partial
// writes); the values come from the sample's own lane by shuffles.  (Blocks are
// whole waves.)  Samples of one key within a span of consecutive samples have
// consecutive ranks, so their records are neighbours: the blocks of a span run on
// one XCD, whose L2 merges those partial-line writes.
__global__ void k_bin_scatter(const double *__restrict__ ptg, int64_t n, BinGeom g, const int *__restrict__ key,
                              const int *__restrict__ rank, const int2 *__restrict__ offs, BinSorted out,
                              const float *__restrict__ y) {
    const int64_t s = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    int pos = -1;
    double fu = 0.0, fv = 0.0, psi = 0.0, yv = 0.0;
    if (valid) {
        int r0, c0;
        anchor_of(ptg, s, g, r0, c0, fu, fv, psi);
        pos = offs[key[s]].x + rank[s];
        if (y) {
            // adjoint layout: (fu, fv as FP32; cos psi) and (sin psi; y, idx)
            double sn, cs;
            sincos(psi, &sn, &cs);
            fu = __longlong_as_double((long long)(((unsigned long long)(unsigned)__float_as_int((float)fv) << 32) |
                                                  (unsigned)__float_as_int((float)fu)));
            fv = cs;
            psi = sn;
            yv = __longlong_as_double((long long)(((unsigned long long)(unsigned)(int)s << 32) |
                                                  (unsigned)__float_as_int(y[s])));
        }
    }
    const int lane = threadIdx.x & 63;
    const int hi = lane & 1;
    double2 *rec2 = (double2 *)out.rec;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int src = (lane >> 1) + 32 * half;  // the wave lane whose sample this lane writes
        const int p = __shfl(pos, src);
        const double su = __shfl(fu, src), sv = __shfl(fv, src), sp = __shfl(psi, src), sy = __shfl(yv, src);
        const int64_t sidx = s - lane + src;
        if (p >= 0) {
            // low half (fu, fv); high half (psi, idx in the low word and pad 0); or the adjoint layout
            const double2 v = hi ? make_double2(sp, y ? sy : __longlong_as_double((long long)(unsigned)sidx))
                                 : make_double2(su, sv);
            rec2[2 * (size_t)p + hi] = v;
        }
    }
}

__global__ void k_bin_items(const int *__restrict__ count, const int2 *__restrict__ offs, int64_t nkeys,
                            int4 *__restrict__ items, int chunk) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    const int c = count[k];
    if (c == 0) return;
    const int2 o = offs[k];
    for (int q = 0; q * chunk < c; ++q) {
        const int cnt = c - q * chunk < chunk ? c - q * chunk : chunk;
        items[o.y + q] = make_int4((int)k, o.x + q * chunk, cnt, 0);
    }
}

template <typename T>
__global__ void k_count_nonfinite(const T *__restrict__ x, int64_t n, int *count) {
    int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += isfinite(x[i]) ? 0 : 1;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void k_zero_words(uint4 *a, int64_t nw) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_zero_bytes(unsigned char *a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

}  // namespace

// Zero a device buffer with a kernel (no memset node if the caller captures a graph).
hipError_t sc_launch_zero(void *dst, size_t bytes, hipStream_t stream) {
    const int64_t nw = (int64_t)(bytes / 16);
    if (nw > 0) hipLaunchKernelGGL(k_zero_words, dim3(2048), dim3(256), 0, stream, (uint4 *)dst, nw);
    const int64_t tail = (int64_t)(bytes - 16 * (size_t)nw);
    if (tail > 0) hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, stream, (unsigned char *)dst + 16 * nw, tail);
    return hipGetLastError();
}

hipError_t sc_launch_count_nonfinite(const void *x, int64_t n, int f32, int *count, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (f32)
        hipLaunchKernelGGL(k_count_nonfinite<float>, dim3((unsigned)nb), dim3(256), 0, stream, (const float *)x, n, count);
    else
        hipLaunchKernelGGL(k_count_nonfinite<double>, dim3((unsigned)nb), dim3(256), 0, stream, (const double *)x, n,
                           count);
    return hipGetLastError();
}

hipError_t sc_launch_binning(sc_plan *p, const double *ptg, int64_t n, const float *y) {
    BinWork &w = p->bw;
    w.last_n = n;
    const BinGeom g = sc_bin_geom(p);
    const int64_t nkeys = (int64_t)g.nkr * g.nkc;
    const int bs = 256;
    const unsigned gs = (unsigned)((n + bs - 1) / bs);
    hipLaunchKernelGGL(k_fill_int, dim3(1024), dim3(256), 0, p->stream, w.count, nkeys, 0);
    const unsigned gk = (unsigned)((n + KEYS_NT * KEYS_SPT - 1) / (KEYS_NT * KEYS_SPT));
    hipLaunchKernelGGL(k_bin_keys, dim3(gk), dim3(KEYS_NT), 0, p->stream, ptg, n, g, w.key, w.rank, w.count);
    const int nblk = (int)((nkeys + SCAN_BLOCK - 1) / SCAN_BLOCK);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(SCAN_NT), 0, p->stream, w.count, nkeys, w.sums, p->bin_chunk);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, p->stream, w.sums, nblk, w.totals);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(SCAN_NT), 0, p->stream, w.count, nkeys, w.sums, w.offs,
                       p->bin_chunk);
    hipLaunchKernelGGL(k_bin_scatter, dim3(gs), dim3(bs), 0, p->stream, ptg, n, g, w.key, w.rank, w.offs, w.sorted, y);
    hipLaunchKernelGGL(k_bin_items, dim3((unsigned)((nkeys + bs - 1) / bs)), dim3(bs), 0, p->stream, w.count,
                       w.offs, nkeys, w.items, p->bin_chunk);
    return hipGetLastError();
}
