// sc_api.cpp -- C ABI of libsidelobe: argument validation, plan geometry and
// workspace, and the order of kernel launches.  No arithmetic of the method
// happens on the host: every stage runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "sc_common.h"

namespace {

thread_local char g_msg[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(SC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Device (or managed) memory of the current HIP context?
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // unregistered host memory: clear the error
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

bool is_smooth(int n) {
    for (int q : {2, 3, 5})
        while (n % q == 0) n /= q;
    return n == 1;
}
int next_smooth(int n, bool even) {
    if (even && (n & 1)) ++n;
    while (!is_smooth(n)) n += even ? 2 : 1;
    return n;
}

// Fewest passes of radix <= 16 (2^x 3^y 5^z) for 2^a 3^b 5^c, by exhaustive
// search over the (small) exponent space; ties keep the first (largest) radix.
static int radix_passes(int a, int b, int c, int *out) {
    if (a == 0 && b == 0 && c == 0) return 0;
    int best = 1 << 20, tmp[SC_MAX_RADICES];
    for (int x = a; x >= 0; --x)
        for (int y = b; y >= 0; --y)
            for (int z = c; z >= 0; --z) {
                int R = 1;
                for (int i = 0; i < x; ++i) R *= 2;
                for (int i = 0; i < y; ++i) R *= 3;
                for (int i = 0; i < z; ++i) R *= 5;
                if (R == 1 || R > 16 || R == 7 || R == 14) continue;
                const int np = 1 + radix_passes(a - x, b - y, c - z, tmp + 1);
                if (np < best && np <= SC_MAX_RADICES) {
                    best = np;
                    tmp[0] = R;
                    for (int i = 0; i < np; ++i) out[i] = tmp[i];
                }
            }
    return best;
}

bool factor_fft(int n, FftPlan *P) {
    P->n = n;
    P->nst = 0;
    if (n < 2 || n > 1024 * 9) return false;  // longest LDS transform: 1024 threads x 9 points
    int m = n, a = 0, b = 0, c = 0;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (m % 5 == 0) { m /= 5; ++c; }
    if (m != 1) return false;
    static const int p540[] = {SC_PLAN_540}, p1080[] = {SC_PLAN_1080}, p2160[] = {SC_PLAN_2160},
                     p4320[] = {SC_PLAN_4320};
    const int *fixed = n == 540 ? p540 : n == 1080 ? p1080 : n == 2160 ? p2160 : n == 4320 ? p4320 : nullptr;
    if (fixed) {
        // the compile-time kernels' order
        for (int prod = 1; prod < n; prod *= fixed[P->nst], ++P->nst) P->r[P->nst] = fixed[P->nst];
    } else {
        int rad[SC_MAX_RADICES];
        const int np = radix_passes(a, b, c, rad);
        // Odd radices first: their strided writes (span 1, R1, ...) do not collide in
        // LDS banks, and by the time the even radices run the span is large, where a
        // pass reads and writes contiguous runs.
        for (int i = 0; i < np; ++i)
            if (rad[i] & 1) P->r[P->nst++] = rad[i];
        for (int i = 0; i < np; ++i)
            if (!(rad[i] & 1)) P->r[P->nst++] = rad[i];
    }
    int ns = 1;
    for (int s = 0; s < P->nst; ++s) {
        P->ns[s] = ns;
        P->tws[s] = n / (ns * P->r[s]);
        P->mag[s] = ns > 1 ? (unsigned)((0x100000000ull + (unsigned long long)ns - 1) / (unsigned long long)ns) : 0u;
        ns *= P->r[s];
    }
    return true;
}

// A transform of length n as P sub-transforms of length n / P that fit one workgroup
// (smallest such P <= 16; P = 1 when the whole transform fits).
bool split_fft(int n, int *P, FftPlan *Q) {
    for (int q = 1; q <= 16; ++q)
        if (n % q == 0 && n / q <= 1024 * 9 && factor_fft(n / q, Q)) {
            *P = q;
            return true;
        }
    return false;
}

// Record the start event of a timed launch; returns the slot or -1.
int timing_begin(sc_plan *p, int stage) {
    if (!p->timing) return -1;
    if (p->tl_n == p->tl_cap) {
        int cap = p->tl_cap ? 2 * p->tl_cap : 64;
        TimedLaunch *n = (TimedLaunch *)std::realloc(p->tl, sizeof(TimedLaunch) * cap);
        if (!n) return -1;
        for (int i = p->tl_cap; i < cap; ++i) {
            n[i].a = nullptr;
            n[i].b = nullptr;
        }
        p->tl = n;
        p->tl_cap = cap;
    }
    TimedLaunch &t = p->tl[p->tl_n];
    if (!t.a && (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess)) return -1;
    t.stage = stage;
    if (hipEventRecord(t.a, p->stream) != hipSuccess) return -1;
    return p->tl_n++;
}
void timing_end(sc_plan *p, int slot) {
    if (slot >= 0) (void)hipEventRecord(p->tl[slot].b, p->stream);
}

// Stream-ordered release: the buffers stay valid for everything already queued
// on `s` and return to the pool when `s` reaches this point (no host wait).
void free_bin_work(BinWork &w, hipStream_t s) {
    void *bufs[] = {w.count, w.offs, w.sums, w.totals, w.key, w.rank, w.sorted.rec, w.items};
    for (void *b : bufs)
        if (b) (void)hipFreeAsync(b, s);
    std::memset(&w, 0, sizeof(w));
}

int alloc(void **dst, size_t bytes, size_t *total);
int alloc_async(void **dst, size_t bytes, size_t *total, hipStream_t s);

// Binning workspace for passes of up to `need` samples (grown on demand).  The
// old buffers are released and the new ones allocated in the order of the plan's
// stream, so work already queued keeps reading the old ones and the host never
// waits for the device here.
int ensure_bin_work(sc_plan *p, int64_t need) {
    BinWork &w = p->bw;
    if (w.cap >= need) return SC_OK;
    if (p->bin_fixed)
        return fail(SC_ESTATE, "plan belongs to a batch: %lld samples exceed its %lld-sample buffers",
                    (long long)need, (long long)w.cap);
    p->ws_bytes -= w.bytes;
    free_bin_work(w, p->stream);
    const BinGeom g = sc_bin_geom(p);
    const int64_t nkeys = (int64_t)g.nkr * g.nkc;
    const int64_t nblk = (nkeys + 4095) / 4096;
    size_t tot = 0;
    int rc = SC_OK;
    hipStream_t s = p->stream;
    rc = rc ? rc : alloc_async((void **)&w.count, sizeof(int) * nkeys, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.offs, sizeof(int2) * nkeys, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.sums, sizeof(int2) * nblk, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.totals, sizeof(int) * 4, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.key, sizeof(int) * need, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.rank, sizeof(int) * need, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.sorted.rec, sizeof(BinRec) * need, &tot, s);
    rc = rc ? rc : alloc_async((void **)&w.items, sizeof(int4) * need, &tot, s);
    if (rc) {
        free_bin_work(w, s);
        return rc;
    }
    w.cap = need;
    w.nkeys = nkeys;
    w.bytes = tot;
    p->ws_bytes += tot;
    return SC_OK;
}

// Release every buffer of a plan (the caller has synchronised its stream; the
// stream-ordered ones are returned on the stream, which the caller then waits for).
void free_plan_buffers(sc_plan *p) {
    free_bin_work(p->bw, p->stream);
    {
        void *pool[] = {p->twpsi, p->gpsi, p->cube};
        for (void *b : pool)
            if (b) (void)hipFreeAsync(b, p->stream);
        p->twpsi = nullptr;
        p->gpsi = nullptr;
        p->cube = nullptr;
    }
    if (p->gmaps) (void)hipFree(p->gmaps);
    if (p->vcount) (void)hipFree(p->vcount);
    if (p->pg) (void)hipFreeAsync(p->pg, p->stream);
    if (p->GA) (void)hipFree(p->GA);
    if (p->GB) (void)hipFree(p->GB);
    p->GB = nullptr;
    p->gmaps = nullptr;
    p->GA = nullptr;
    for (int i = 0; i < p->tl_cap; ++i) {
        if (p->tl[i].a) (void)hipEventDestroy(p->tl[i].a);
        if (p->tl[i].b) (void)hipEventDestroy(p->tl[i].b);
    }
    std::free(p->tl);
    p->tl = nullptr;
    p->tl_cap = p->tl_n = 0;
    void *bufs[] = {p->F, p->G, p->maps, p->rroot, p->sbin_m, p->sbin_e, p->rtab, p->tw2, p->tw2os, p->twphi,
                    p->phase, p->dphi, p->glx, p->glw, p->S, p->ctab, p->ctab_off};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

// Test hook: SC_FAIL_ALLOC_AFTER=k makes every allocation after the first k of the
// process fail (read once), so tests can check that a failed allocation returns
// SC_ENOMEM and releases what was already allocated.
bool injected_alloc_failure() {
    static const long long limit = [] {
        const char *v = std::getenv("SC_FAIL_ALLOC_AFTER");
        return v ? std::atoll(v) : -1LL;
    }();
    static std::atomic<long long> count{0};
    return limit >= 0 && count.fetch_add(1) >= limit;
}

int alloc(void **dst, size_t bytes, size_t *total) {
    hipError_t e = injected_alloc_failure() ? hipErrorOutOfMemory : hipMalloc(dst, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    *total += bytes;
    return SC_OK;
}

// Stream-ordered allocation (usable by work queued on `s` after this call, and by
// other streams ordered after it).
int alloc_async(void **dst, size_t bytes, size_t *total, hipStream_t s) {
    hipError_t e = injected_alloc_failure() ? hipErrorOutOfMemory : hipMallocAsync(dst, bytes, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SC_ENOMEM, "hipMallocAsync(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    *total += bytes;
    return SC_OK;
}

// Make `next` wait for everything queued so far on the plan's stream, then enqueue
// the plan's later work on `next`.
int switch_stream(sc_plan *p, hipStream_t next) {
    if (next == p->stream) return SC_OK;
    hipError_t e = hipSuccess;
    if (!p->ev_stream) e = hipEventCreateWithFlags(&p->ev_stream, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p->ev_stream, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, p->ev_stream, 0);
    if (e != hipSuccess) return hip_fail(e, "ordering the new stream after the plan's stream");
    p->stream = next;
    return SC_OK;
}

struct AttrCache {
    std::mutex mu;
    std::map<const void *, size_t> lds;
    std::map<std::tuple<const void *, int, size_t, int, int>, int> grid;
};
AttrCache &attr_cache() {
    static AttrCache *c = new AttrCache();
    return *c;
}

struct PlanCache {
    std::mutex mu;
    std::map<std::tuple<int, int, int, int>, sc_plan *> plans;
};
PlanCache &plan_cache() {
    static PlanCache *c = new PlanCache();  // never destroyed: plans outlive static teardown
    return *c;
}

}  // namespace

hipError_t sc_set_lds_attr(const void *kern, size_t lds) {
    AttrCache &c = attr_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.lds.find(kern);
    if (it != c.lds.end() && it->second >= lds) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) c.lds[kern] = lds;
    return e;
}

int sc_persistent_grid(const void *kern, int block, size_t lds, int wgs_per_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    AttrCache &c = attr_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto key = std::make_tuple(kern, block, lds, wgs_per_cu, dev);
    auto it = c.grid.find(key);
    if (it != c.grid.end()) return it->second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    if (per_cu < 1) per_cu = 1;
    if (wgs_per_cu > 0 && wgs_per_cu < per_cu) per_cu = wgs_per_cu;
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu < 1) ncu = 256;
    c.grid[key] = per_cu * ncu;
    return per_cu * ncu;
}

// Validation mode (SC_PARAM_VALIDATE): count the NaN / infinite values of an input
// on the plan's stream and wait for the count; SC_EINVAL names the input.  Off by
// default: then nothing is inspected and a NaN angle is read as 0.
static int validate_input(sc_plan *p, const char *what, const void *x, int64_t n, int f32) {
    if (!p->validate || n <= 0) return SC_OK;
    if (!p->vcount) {
        size_t tot = 0;
        const int rc = alloc((void **)&p->vcount, sizeof(int), &tot);
        if (rc) return rc;
    }
    int count = 0;
    hipError_t e = sc_launch_zero(p->vcount, sizeof(int), p->stream);
    if (e == hipSuccess) e = sc_launch_count_nonfinite(x, n, f32, p->vcount, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&count, p->vcount, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "input validation");
    if (count) return fail(SC_EINVAL, "%s holds %d NaN or infinite values (validation mode)", what, count);
    return SC_OK;
}

static int64_t n_blm_values(const sc_plan *p) {  // doubles in the beam layout
    return 2 * ((int64_t)(p->kmax + 1) * (p->lmax + 1) - (int64_t)p->kmax * (p->kmax + 1) / 2);
}
static int64_t n_alm_values(const sc_plan *p) {  // doubles in the sky layout
    return (int64_t)(p->alm_lmax + 1) * (p->alm_lmax + 2);
}

int sc_psi_slack_bytes();  // k_psi.hip: zeroed bytes after the cube
hipError_t sc_launch_gather_psi_sorted(sc_plan *p, const double *ptg, int64_t n, void *tod);  // k_psi.hip

extern "C" {

const char *sc_strerror(int code) {
    switch (code) {
        case SC_OK: return "success";
        case SC_EINVAL: return "invalid argument";
        case SC_ENOMEM: return "out of device memory";
        case SC_EHIP: return "HIP runtime error";
        case SC_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

const char *sc_last_error(void) { return g_msg; }

int sc_plan_create(sc_plan **out, int lmax, int kmax, int precision, int kernel_width, void *stream) {
    g_msg[0] = 0;
    if (!out) return fail(SC_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    if (lmax < 0) return fail(SC_EINVAL, "lmax = %d < 0", lmax);
    if (lmax > SC_LMAX_MAX) return fail(SC_EINVAL, "lmax = %d above the supported %d", lmax, SC_LMAX_MAX);
    if (kmax < 0 || kmax > lmax) return fail(SC_EINVAL, "kmax = %d outside [0, lmax = %d]", kmax, lmax);
    if (kmax > 127) return fail(SC_EINVAL, "kmax = %d above the supported 127", kmax);
    if (precision != SC_FP64 && precision != SC_F64MAPS_F32GATHER && precision != SC_MIXED)
        return fail(SC_EINVAL, "unknown precision %d", precision);
    int W = kernel_width;
    if (W == 0) W = precision == SC_FP64 ? 14 : 8;
    if (W < 4 || W > 16 || (W & 1)) return fail(SC_EINVAL, "kernel width %d not an even number in [4, 16]", W);

    sc_plan *p = new (std::nothrow) sc_plan;
    if (!p) return fail(SC_ENOMEM, "host allocation failed");
    std::memset(p, 0, sizeof(*p));
    p->lmax = lmax;
    p->kmax = kmax;
    p->prec = precision;
    p->W = W;
    p->beta = 2.30 * W;  // exponential-of-semicircle shape for 2x oversampling
    p->stream = (hipStream_t)stream;
    // theta: 2 nring >= 2 lmax + 2 samples of the full circle represent a degree-lmax
    // trigonometric polynomial exactly; the fine grid oversamples it >= 2x.
    p->n2 = next_smooth(2 * lmax + 2, true);
    p->nring = p->n2 / 2;
    p->n2os = next_smooth(2 * p->n2, true);
    // every kept row (n2os / 2 + W of them) on its own grid index
    if (p->n2os < 2 * W) p->n2os = next_smooth(2 * W, true);
    p->nphi = next_smooth(2 * (2 * lmax + 1), false);
    if (p->nphi < 2 * W) p->nphi = next_smooth(2 * W, false);
    p->rows = p->n2os / 2 + W;
    p->cols = p->nphi + W - 1;
    // component pairs: (2k, 2k + 1) hold the cos k psi and sin k psi maps; the
    // sin 0 psi slot (component 1) is zero, so each phi column stores one pair.
    p->ncomp = 2 * kmax + 2;
    // FP32 maps: components padded to the 16-wide tiles of the matrix-core gather
    // (and a whole number of four-component groups of the column-tiled storage);
    // FP64 maps: to 4 (whole two-component groups).
    p->ncp = precision == SC_FP64 ? (p->ncomp + 3) & ~3 : (p->ncomp + 15) & ~15;
    p->nq = 128;
    p->alm_lmax = lmax;
    p->bin_chunk = BIN_CHUNK;
    p->gather_wgs_per_cu = 0;
    p->gather_waves = 4;
    p->gather_mma = SC_MMA_SPLIT16;
    {
        const char *g = std::getenv("SC_GATHER_PATH");
        p->gather_direct = (g && std::strcmp(g, "direct") == 0) ? 1 : 0;
        p->gather_valu = (g && std::strcmp(g, "valu") == 0) ? 1 : 0;
        const char *b = std::getenv("SC_BIN_PASS_MAX");
        long long v = b ? std::atoll(b) : 0;
        p->bin_pass_max = (v > 0 && v < BIN_PASS_MAX) ? (int64_t)v : (int64_t)BIN_PASS_MAX;
    }
    sc_choose_ring_layout(p->nring, &p->rpt, &p->ngroups);
    sc_choose_ring_layout_mixed(p->nring, &p->rpt_mx, &p->ngroups_mx);
    if (!split_fft(p->n2, &p->sp2, &p->p2) || !split_fft(p->n2os, &p->spos, &p->p2os) ||
        !split_fft(p->nphi, &p->spphi, &p->pphi)) {
        delete p;
        return fail(SC_EINVAL, "lmax = %d: no transform plan for lengths %d, %d, %d", lmax, p->n2, p->n2os, p->nphi);
    }
    p->big = p->sp2 > 1 || p->spos > 1 || p->spphi > 1;
    p->spad = (2 * lmax + 1 + 63) & ~63;
    p->mid32 = precision != SC_FP64 && !p->big;
    p->gst = p->mid32 ? 2 * lmax + 2 : 2 * lmax + 1;

    const size_t nm = 2 * (size_t)lmax + 1;
    size_t tot = 0;
    int rc = SC_OK;
    rc = rc ? rc : alloc((void **)&p->F, sizeof(double2) * (kmax + 1) * nm * p->nring, &tot);
    rc = rc ? rc : alloc((void **)&p->G, sizeof(double2) * (kmax + 1) * (size_t)p->rows * nm, &tot);
    rc = rc ? rc : alloc(&p->maps, sc_map_bytes(p), &tot);
    rc = rc ? rc : alloc((void **)&p->rroot, sizeof(double2) * (size_t)(lmax + 1) * (lmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->sbin_m, sizeof(double) * (lmax + 1) * (kmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->sbin_e, sizeof(int) * (lmax + 1) * (kmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->rtab, sizeof(double) * 5 * p->nring, &tot);
    rc = rc ? rc : alloc((void **)&p->tw2, sizeof(double2) * p->p2.n, &tot);
    rc = rc ? rc : alloc((void **)&p->tw2os, sizeof(double2) * p->p2os.n, &tot);
    rc = rc ? rc : alloc((void **)&p->twphi, sizeof(double2) * p->pphi.n, &tot);
    if (p->big) rc = rc ? rc : alloc((void **)&p->S, sizeof(double2) * (kmax + 1) * nm * (size_t)p->spad, &tot);
    rc = rc ? rc : alloc((void **)&p->phase, sizeof(double2) * nm, &tot);
    rc = rc ? rc : alloc((void **)&p->dphi, sizeof(double) * (lmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->glx, sizeof(double) * p->nq, &tot);
    rc = rc ? rc : alloc((void **)&p->glw, sizeof(double) * p->nq, &tot);
    // Recursion coefficients of every (m, k, l) column for the ring-sum kernels (32 B per
    // entry: 0.66 GB at lmax 512 / kmax 100, 3.2 GB at lmax 8192 / kmax 2); above 8 GiB the
    // kernels compute them per chunk instead.
    std::vector<long long> coff((size_t)(lmax + 1) * (kmax + 1));
    long long ctot = 0;
    for (int m = 0; m <= lmax; ++m)
        for (int k = 0; k <= kmax; ++k) {
            coff[(size_t)m * (kmax + 1) + k] = ctot;
            ctot += lmax - (m > k ? m : k) + 1;
        }
    if ((double)ctot * 32.0 <= 8.0 * (1 << 30)) {
        rc = rc ? rc : alloc((void **)&p->ctab, 32 * (size_t)ctot, &tot);
        rc = rc ? rc : alloc((void **)&p->ctab_off, sizeof(long long) * coff.size(), &tot);
    }
    if (rc) {
        free_plan_buffers(p);
        delete p;
        return rc;
    }
    p->ws_bytes = tot;
    // padding components stay zero for the plan's lifetime
    hipError_t e = hipMemsetAsync(p->maps, 0, sc_map_bytes(p), p->stream);
    if (e == hipSuccess) e = sc_launch_tables(p);
    if (e == hipSuccess && p->ctab)
        e = hipMemcpyAsync(p->ctab_off, coff.data(), sizeof(long long) * coff.size(), hipMemcpyHostToDevice,
                           p->stream);  // coff outlives the synchronisation below
    if (e == hipSuccess) e = sc_launch_rec_table(p);
    if (e == hipSuccess) {
        // ring table in extended host precision: theta_j = (j + 1/2) pi / nring;
        // 1 - cos(theta_j) as 2 sin^2(theta_j / 2), which keeps its full relative
        // precision next to the poles
        std::vector<double> rt(5 * (size_t)p->nring);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int j = 0; j < p->nring; ++j) {
            const long double th = ((long double)j + 0.5L) * pi / (long double)p->nring;
            const long double lc = log2l(cosl(0.5L * th)), ls = log2l(sinl(0.5L * th));
            const long double sh = sinl(0.5L * th);
            rt[5 * j] = (double)(2.0L * sh * sh);
            rt[5 * j + 1] = (double)lc;
            rt[5 * j + 2] = (double)(lc - (long double)(double)lc);
            rt[5 * j + 3] = (double)ls;
            rt[5 * j + 4] = (double)(ls - (long double)(double)ls);
        }
        e = hipMemcpyAsync(p->rtab, rt.data(), sizeof(double) * rt.size(), hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // rt is a local buffer
    }
    if (e != hipSuccess) {
        free_plan_buffers(p);
        delete p;
        return hip_fail(e, "plan table setup");
    }
    *out = p;
    return SC_OK;
}

int sc_plan_destroy(sc_plan *p) {
    if (!p) return SC_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (p->side) {
        const hipError_t es = hipStreamSynchronize(p->side);
        if (e == hipSuccess) e = es;
        (void)hipStreamDestroy(p->side);
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->ev_stream) (void)hipEventDestroy(p->ev_stream);
    free_plan_buffers(p);
    const hipError_t ef = hipStreamSynchronize(p->stream);  // the stream-ordered frees
    if (e == hipSuccess) e = ef;
    delete p;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize in sc_plan_destroy");
    return SC_OK;
}

int sc_plan_set_stream(sc_plan *p, void *stream) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    return switch_stream(p, (hipStream_t)stream);
}

int sc_plan_info(const sc_plan *p, int64_t *out, int nout) {
    if (!p || (nout > 0 && !out)) return fail(SC_EINVAL, "NULL plan or output");
    const int64_t v[] = {p->lmax, p->kmax, p->prec, p->W, p->nring, p->n2, p->n2os, p->nphi,
                         p->rows, p->cols, p->ncomp, p->ncp, (int64_t)p->ws_bytes, p->mid32 ? 8 : 16};
    const int nv = (int)(sizeof(v) / sizeof(v[0]));
    for (int i = 0; i < nout && i < nv; ++i) out[i] = v[i];
    return nv;
}

int sc_set_sky_beam(sc_plan *p, const double *alm, const double *blm) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (!is_device_ptr(alm)) return fail(SC_EINVAL, "alm is not device memory");
    if (!is_device_ptr(blm)) return fail(SC_EINVAL, "blm is not device memory");
    if (((uintptr_t)alm & 15) || ((uintptr_t)blm & 15)) return fail(SC_EINVAL, "alm/blm not 16-byte aligned");
    int rc = validate_input(p, "alm", alm, n_alm_values(p), 0);
    if (!rc) rc = validate_input(p, "blm", blm, n_blm_values(p), 0);
    if (rc) return rc;
    int slot = timing_begin(p, SC_STAGE_RING);
    hipError_t e = p->prec == SC_MIXED ? sc_launch_ring_sums_mixed(p, alm, blm) : sc_launch_ring_sums(p, alm, blm);
    timing_end(p, slot);
    if (e == hipSuccess) {
        slot = timing_begin(p, SC_STAGE_THETA);
        e = sc_launch_theta_upsample(p);
        timing_end(p, slot);
    }
    if (e == hipSuccess) {
        slot = timing_begin(p, SC_STAGE_PHI);
        e = sc_launch_phi_synthesis(p);
        timing_end(p, slot);
    }
    if (e != hipSuccess) return hip_fail(e, "map synthesis launch");
    p->have_maps = 1;
    p->have_cube = 0;  // a cube holds the previous maps
    return SC_OK;
}

// Argument checks of an interpolation (n > 0).
static int check_interp_args(sc_plan *p, const double *ptg, void *tod) {
    if (!is_device_ptr(ptg)) return fail(SC_EINVAL, "ptg is not device memory");
    if (!is_device_ptr(tod)) return fail(SC_EINVAL, "tod is not device memory");
    if (((uintptr_t)ptg & 7) || ((uintptr_t)tod & (p->prec == SC_FP64 ? 7 : 3)))
        return fail(SC_EINVAL, "ptg/tod misaligned");
    return SC_OK;
}

static bool uses_binning(const sc_plan *p) { return !p->gather_direct && sc_gather_binned_supported(p); }

}  // extern "C"

// Library-internal helpers for the other host sources.
int sc_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}
int sc_hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
void sc_clear_error() { g_msg[0] = 0; }
int sc_check_interp_args(sc_plan *p, const double *ptg, void *tod) { return check_interp_args(p, ptg, tod); }
bool sc_uses_binning(const sc_plan *p) { return uses_binning(p); }

extern "C" {

// Binning pass of samples [off, off + cnt) on the plan's current stream.
static int bin_pass(sc_plan *p, const double *ptg, int64_t off, int64_t cnt) {
    const int slot = timing_begin(p, SC_STAGE_BIN);
    const hipError_t e = sc_launch_binning(p, ptg + 3 * off, cnt);
    timing_end(p, slot);
    return e != hipSuccess ? hip_fail(e, "binning launch") : SC_OK;
}

// Binned interpolation in passes; the first pass's binning has already been
// issued when first_binned is set.
static int interpolate_passes(sc_plan *p, const double *ptg, int64_t n, void *tod, bool first_binned) {
    const int64_t pass = n < p->bin_pass_max ? n : p->bin_pass_max;
    const size_t esz = p->prec == SC_FP64 ? 8 : 4;
    for (int64_t off = 0; off < n; off += pass) {
        const int64_t cnt = n - off < pass ? n - off : pass;
        if (off > 0 || !first_binned) {
            const int rc = bin_pass(p, ptg, off, cnt);
            if (rc) return rc;
        }
        const int slot = timing_begin(p, SC_STAGE_GATHER);
        const hipError_t e = sc_launch_gather_binned(p, (char *)tod + esz * off);
        timing_end(p, slot);
        if (e != hipSuccess) return hip_fail(e, "binned gather launch");
    }
    return SC_OK;
}

int sc_interpolate(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (n == 0) return SC_OK;
    if (!p->have_maps) return fail(SC_ESTATE, "sc_interpolate before sc_set_sky_beam");
    int rc = check_interp_args(p, ptg, tod);
    if (!rc) rc = validate_input(p, "ptg", ptg, 3 * n, 0);
    if (rc) return rc;
    if (!uses_binning(p)) {
        int slot = timing_begin(p, SC_STAGE_GATHER);
        hipError_t e = sc_launch_gather(p, ptg, n, tod);
        timing_end(p, slot);
        if (e != hipSuccess) return hip_fail(e, "gather launch");
        return SC_OK;
    }
    rc = ensure_bin_work(p, n < p->bin_pass_max ? n : p->bin_pass_max);
    if (rc) return rc;
    return interpolate_passes(p, ptg, n, tod, false);
}

// Free the psi cube and its tables (kept until the grid size changes), in the
// order of the plan's stream: earlier work may still read them.
static void free_psi(sc_plan *p) {
    void *bufs[] = {p->twpsi, p->gpsi, p->cube};
    for (void *b : bufs)
        if (b) (void)hipFreeAsync(b, p->stream);
    p->twpsi = nullptr;
    p->gpsi = nullptr;
    p->cube = nullptr;
    p->npsi = p->npst = 0;
    p->have_cube = 0;
}

int sc_plan_build_psi_cube(sc_plan *p, int npsi) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (!p->have_maps) return fail(SC_ESTATE, "sc_plan_build_psi_cube before sc_set_sky_beam");
    int lo = 2 * (2 * p->kmax + 1);
    if (lo < 2 * p->W) lo = 2 * p->W;
    if (npsi == 0) npsi = next_smooth(lo, false);
    if (npsi < lo || npsi > sc_psi_max_len() || !is_smooth(npsi))
        return fail(SC_EINVAL, "npsi = %d: needs a product of 2, 3, 5 in [%d, %d]", npsi, lo, sc_psi_max_len());
    if (npsi != p->npsi) {
        free_psi(p);
        FftPlan P;
        if (!factor_fft(npsi, &P)) return fail(SC_EINVAL, "npsi = %d has no transform plan", npsi);
        const int npst = (npsi + p->W - 1 + 3) & ~3;
        const size_t bytes = sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * npst;
        size_t tot = 0;
        int rc = alloc_async((void **)&p->twpsi, sizeof(double2) * npsi, &tot, p->stream);
        rc = rc ? rc : alloc_async((void **)&p->gpsi, sizeof(double) * (p->kmax + 1), &tot, p->stream);
        rc = rc ? rc : alloc_async(&p->cube, bytes + sc_psi_slack_bytes(), &tot, p->stream);  // + the gather's zeroed slack
        if (rc) {
            free_psi(p);
            return rc;
        }
        p->npsi = npsi;
        p->npst = npst;
        p->ppsi = P;
        const hipError_t e = sc_launch_psi_tables(p);
        if (e != hipSuccess) {
            free_psi(p);
            return hip_fail(e, "psi table launch");
        }
    }
    const hipError_t e = sc_launch_psi_cube(p);
    if (e != hipSuccess) return hip_fail(e, "psi cube launch");
    p->have_cube = 1;
    return SC_OK;
}

int sc_interpolate_psi(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (n == 0) return SC_OK;
    if (!p->have_cube) return fail(SC_ESTATE, "sc_interpolate_psi without a cube of the current maps");
    int rc = check_interp_args(p, ptg, tod);
    if (!rc) rc = validate_input(p, "ptg", ptg, 3 * n, 0);
    if (rc) return rc;
    if (p->prec == SC_FP64 || !uses_binning(p)) {
        const hipError_t e = sc_launch_gather_psi(p, ptg, n, tod);
        return e != hipSuccess ? hip_fail(e, "psi gather launch") : SC_OK;
    }
    // FP32 cube: samples in anchor order (the binning of the two-dimensional gather), in passes
    const int64_t pass = n < p->bin_pass_max ? n : p->bin_pass_max;
    rc = ensure_bin_work(p, pass);
    if (rc) return rc;
    for (int64_t off = 0; off < n; off += pass) {
        const int64_t cnt = n - off < pass ? n - off : pass;
        rc = bin_pass(p, ptg, off, cnt);
        if (rc) return rc;
        const hipError_t e = sc_launch_gather_psi_sorted(p, ptg + 3 * off, cnt, (float *)tod + off);
        if (e != hipSuccess) return hip_fail(e, "psi gather launch");
    }
    return SC_OK;
}

int sc_plan_convolve(sc_plan *p, const double *alm, const double *blm, const double *ptg, int64_t n, void *tod) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (n == 0 || !uses_binning(p)) {
        const int rc = sc_set_sky_beam(p, alm, blm);
        return rc ? rc : sc_interpolate(p, ptg, n, tod);
    }
    int rc = check_interp_args(p, ptg, tod);
    if (!rc && p->validate) {
        if (!is_device_ptr(alm) || !is_device_ptr(blm)) return fail(SC_EINVAL, "alm/blm is not device memory");
        rc = validate_input(p, "alm", alm, n_alm_values(p), 0);
        if (!rc) rc = validate_input(p, "blm", blm, n_blm_values(p), 0);
        if (!rc) rc = validate_input(p, "ptg", ptg, 3 * n, 0);
    }
    if (rc) return rc;
    rc = ensure_bin_work(p, n < p->bin_pass_max ? n : p->bin_pass_max);
    if (rc) return rc;
    if (!p->side) {
        hipError_t e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "side stream setup");
    }
    // The first binning pass depends only on the pointings: it runs on the side
    // stream (after everything queued so far on the plan's stream, which may still
    // read the binning buffers) while the maps are synthesised.
    hipStream_t main = p->stream;
    hipError_t e = hipEventRecord(p->ev_fork, main);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "stream fork");
    p->stream = p->side;
    rc = bin_pass(p, ptg, 0, n < p->bin_pass_max ? n : p->bin_pass_max);
    p->stream = main;
    e = hipEventRecord(p->ev_join, p->side);
    if (rc == SC_OK && e != hipSuccess) rc = hip_fail(e, "stream join");
    const int rs = sc_set_sky_beam(p, alm, blm);
    // join before anything else can fail, so the side stream never runs ahead of a
    // later call's use of the binning buffers
    e = hipStreamWaitEvent(main, p->ev_join, 0);
    if (rc) return rc;
    if (rs) return rs;
    if (e != hipSuccess) return hip_fail(e, "stream join");
    return interpolate_passes(p, ptg, n, tod, true);
}

int sc_convolve(const double *alm, const double *blm, int lmax, int kmax, const double *ptg, int64_t n, void *tod,
                int precision, void *stream) {
    g_msg[0] = 0;
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    PlanCache &pc = plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    auto key = std::make_tuple(lmax, kmax, precision, dev);
    sc_plan *p = nullptr;
    auto it = pc.plans.find(key);
    if (it == pc.plans.end()) {
        int rc = sc_plan_create(&p, lmax, kmax, precision, 0, stream);
        if (rc) return rc;
        pc.plans[key] = p;
    } else {
        p = it->second;
        // the cached plan's buffers may still be in use by work on another stream
        const int rc = switch_stream(p, (hipStream_t)stream);
        if (rc) return rc;
    }
    return sc_plan_convolve(p, alm, blm, ptg, n, tod);
}

int sc_convolve_release_cache(void) {
    g_msg[0] = 0;
    PlanCache &pc = plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    int rc = SC_OK;
    for (auto &kv : pc.plans) {
        const int r = sc_plan_destroy(kv.second);
        if (r && rc == SC_OK) rc = r;
    }
    pc.plans.clear();
    return rc;
}

int sc_dipole_response(const double *blm, int lmax, int kmax, const double *ptg, int64_t n, const double *beta,
                       int64_t samples_per_period, double T0, double q, double *out, void *stream) {
    g_msg[0] = 0;
    if (lmax < 0 || kmax < 0 || kmax > lmax) return fail(SC_EINVAL, "lmax = %d, kmax = %d", lmax, kmax);
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (samples_per_period < 1) return fail(SC_EINVAL, "samples_per_period = %lld < 1", (long long)samples_per_period);
    if (n == 0) return SC_OK;
    if (!is_device_ptr(blm) || !is_device_ptr(ptg) || !is_device_ptr(beta) || !is_device_ptr(out))
        return fail(SC_EINVAL, "blm/ptg/beta/out must be device memory");
    if (((uintptr_t)blm & 15) || ((uintptr_t)ptg & 7) || ((uintptr_t)beta & 7) || ((uintptr_t)out & 7))
        return fail(SC_EINVAL, "blm/ptg/beta/out misaligned");
    const hipError_t e = sc_launch_dipole(blm, lmax, kmax, ptg, n, beta, samples_per_period, T0, q, out,
                                          (hipStream_t)stream);
    return e != hipSuccess ? hip_fail(e, "dipole launch") : SC_OK;
}

// Component tiles of the scatter kernels' instantiation (the tile count rounded up to
// 1, 2, 3, 5, 9, 13 or 16): the patch gradients of the deterministic mode hold 16 of
// them per tile.
static int scatter_tiles(const sc_plan *p) {
    const int ct = (p->ncomp + 15) / 16;
    return ct <= 3 ? ct : ct <= 5 ? 5 : ct <= 9 ? 9 : ct <= 13 ? 13 : 16;
}

// The part of the adjoint that depends on neither coefficient set: scatter of the
// TOD gradient onto gradient maps, then the adjoint phi and theta transforms
// (ring-sum gradients in p->F).
static int adjoint_to_rings(sc_plan *p, const double *ptg, const void *tod_grad, int64_t n) {
    const size_t map_bytes = sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp;
    const size_t nalm = (size_t)(p->lmax + 1) * (p->lmax + 2) / 2;
    if (!p->gmaps) {
        size_t tot = 0;
        int rc = alloc(&p->gmaps, map_bytes, &tot);
        if (!rc) rc = alloc((void **)&p->GA, sizeof(double2) * (p->kmax + 1) * nalm * sc_adjoint_slabs(p), &tot);
        if (rc) {
            if (p->gmaps) (void)hipFree(p->gmaps);
            p->gmaps = nullptr;
            return rc;
        }
        p->adj_bytes = tot;
        p->ws_bytes += tot;
    }
    int slot = timing_begin(p, SC_STAGE_SCATTER);
    hipError_t e = sc_launch_zero(p->gmaps, map_bytes, p->stream);
    timing_end(p, slot);
    if (e != hipSuccess) return hip_fail(e, "gradient map clear");
    if (n > 0) {
        if (sc_scatter_binned_supported(p)) {
            const int64_t pass = n < p->bin_pass_max ? n : p->bin_pass_max;
            int rc = ensure_bin_work(p, pass);
            if (rc) return rc;
            // The deterministic mode bins every anchor into one work item (restored below)
            // and orders its samples by index; a pass whose largest anchor exceeds what
            // the ordering kernel holds is binned again in smaller passes.
            struct ChunkGuard {
                sc_plan *p;
                int saved;
                ~ChunkGuard() { p->bin_chunk = saved; }
            } guard{p, p->bin_chunk};
            if (p->det_adjoint) p->bin_chunk = 1 << 30;
            int64_t cur = pass;
            for (int64_t off = 0; off < n;) {
                const int64_t cnt = n - off < cur ? n - off : cur;
                slot = timing_begin(p, SC_STAGE_BIN);
                // the records carry the pass's TOD gradient (binned scatter: FP32 forms only)
                e = sc_launch_binning(p, ptg + 3 * off, cnt, (const float *)tod_grad + off);
                timing_end(p, slot);
                if (e != hipSuccess) return hip_fail(e, "binning launch");
                if (p->det_adjoint) {
                    // work-item count and largest item are read back (the mode waits for the binning)
                    int nitems = 0, maxn = 0;
                    e = hipMemcpyAsync(&nitems, p->bw.totals + 1, sizeof(int), hipMemcpyDeviceToHost, p->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
                    if (e == hipSuccess) e = sc_launch_zero(p->bw.totals + 3, sizeof(int), p->stream);
                    if (e == hipSuccess) e = sc_launch_det_order(p, nitems);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(&maxn, p->bw.totals + 3, sizeof(int), hipMemcpyDeviceToHost, p->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
                    if (e != hipSuccess) return hip_fail(e, "deterministic ordering");
                    if (maxn > sc_det_max_items()) {
                        // a pass of at most that many samples always fits; shrink and bin again
                        const int64_t next = cnt * sc_det_max_items() / (2 * (int64_t)maxn);
                        cur = next > 0 ? next : 1;
                        continue;
                    }
                    const size_t need = sizeof(float) * (size_t)nitems * 64 * 16 * (size_t)scatter_tiles(p);
                    if (need > p->pg_bytes) {
                        if (p->pg) (void)hipFreeAsync(p->pg, p->stream);
                        p->pg = nullptr;
                        p->ws_bytes -= p->pg_bytes;
                        p->pg_bytes = 0;
                        size_t tot = 0;
                        const int rc2 = alloc_async((void **)&p->pg, need, &tot, p->stream);
                        if (rc2) return rc2;
                        p->ws_bytes += need;
                        p->pg_bytes = need;
                    }
                }
                slot = timing_begin(p, SC_STAGE_SCATTER);
                e = sc_launch_scatter_binned(p, p->gmaps);
                if (e == hipSuccess && p->det_adjoint) e = sc_launch_scatter_reduce(p, p->gmaps);
                timing_end(p, slot);
                if (e != hipSuccess) return hip_fail(e, "binned scatter launch");
                off += cnt;
            }
        } else {
            slot = timing_begin(p, SC_STAGE_SCATTER);
            e = sc_launch_scatter(p, ptg, n, tod_grad, p->gmaps);
            timing_end(p, slot);
            if (e != hipSuccess) return hip_fail(e, "scatter launch");
        }
    }
    slot = timing_begin(p, SC_STAGE_ADJ_FFT);
    e = sc_launch_phi_adjoint(p, p->gmaps);
    if (e == hipSuccess) e = sc_launch_theta_adjoint(p);
    timing_end(p, slot);
    if (e != hipSuccess) return hip_fail(e, "adjoint transform launch");
    return SC_OK;
}

static int check_adjoint_args(sc_plan *p, const double *coefs, const double *ptg, const void *tod_grad, int64_t n,
                              double *grad) {
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (!is_device_ptr(coefs)) return fail(SC_EINVAL, "coefficients are not device memory");
    if (!is_device_ptr(grad)) return fail(SC_EINVAL, "gradient output is not device memory");
    if (n > 0 && (!is_device_ptr(ptg) || !is_device_ptr(tod_grad)))
        return fail(SC_EINVAL, "ptg/tod_grad is not device memory");
    if (((uintptr_t)coefs & 15) || ((uintptr_t)grad & 15)) return fail(SC_EINVAL, "coefficients/gradient not 16-byte aligned");
    if (n > 0 && (((uintptr_t)ptg & 7) || ((uintptr_t)tod_grad & (p->prec == SC_FP64 ? 7 : 3))))
        return fail(SC_EINVAL, "ptg/tod_grad misaligned");
    return SC_OK;
}

int sc_convolve_adjoint(sc_plan *p, const double *blm, const double *ptg, const void *tod_grad, int64_t n,
                        double *alm_grad) {
    g_msg[0] = 0;
    int rc = check_adjoint_args(p, blm, ptg, tod_grad, n, alm_grad);
    if (!rc) rc = validate_input(p, "blm", blm, n_blm_values(p), 0);
    if (!rc) rc = validate_input(p, "ptg", ptg, 3 * n, 0);
    if (!rc) rc = validate_input(p, "tod_grad", tod_grad, n, p->prec != SC_FP64);
    if (rc) return rc;
    rc = adjoint_to_rings(p, ptg, tod_grad, n);
    if (rc) return rc;
    const int slot = timing_begin(p, SC_STAGE_ADJ_RING);
    const hipError_t e = sc_launch_ring_sums_adjoint(p, blm, alm_grad);
    timing_end(p, slot);
    if (e != hipSuccess) return hip_fail(e, "adjoint ring-sum launch");
    return SC_OK;
}

int sc_convolve_adjoint_beam(sc_plan *p, const double *alm, const double *ptg, const void *tod_grad, int64_t n,
                             double *blm_grad) {
    g_msg[0] = 0;
    int rc = check_adjoint_args(p, alm, ptg, tod_grad, n, blm_grad);
    if (!rc) rc = validate_input(p, "alm", alm, n_alm_values(p), 0);
    if (!rc) rc = validate_input(p, "ptg", ptg, 3 * n, 0);
    if (!rc) rc = validate_input(p, "tod_grad", tod_grad, n, p->prec != SC_FP64);
    if (rc) return rc;
    if (!p->GB) {
        const size_t nblm = (size_t)(p->kmax + 1) * (2 * p->lmax + 2 - p->kmax) / 2;
        size_t tot = 0;
        rc = alloc((void **)&p->GB, sizeof(double2) * (size_t)(p->lmax + 1) * nblm * sc_adjoint_slabs(p), &tot);
        if (rc) return rc;
        p->adj_bytes += tot;
        p->ws_bytes += tot;
    }
    rc = adjoint_to_rings(p, ptg, tod_grad, n);
    if (rc) return rc;
    const int slot = timing_begin(p, SC_STAGE_ADJ_RING);
    const hipError_t e = sc_launch_ring_sums_adjoint_beam(p, alm, blm_grad);
    timing_end(p, slot);
    if (e != hipSuccess) return hip_fail(e, "beam adjoint ring-sum launch");
    return SC_OK;
}

int sc_plan_set_param(sc_plan *p, int param, int64_t v) {
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    switch (param) {
        case SC_PARAM_BIN_CHUNK:
            if (v < 16 || v > (1 << 20)) return fail(SC_EINVAL, "bin chunk %lld outside [16, 2^20]", (long long)v);
            p->bin_chunk = (int)v;
            return SC_OK;
        case SC_PARAM_GATHER_WGS_PER_CU:
            if (v < 0 || v > 16) return fail(SC_EINVAL, "workgroups per CU %lld outside [0, 16]", (long long)v);
            p->gather_wgs_per_cu = (int)v;
            return SC_OK;
        case SC_PARAM_GATHER_WAVES:
            if (v != 4 && v != 8) return fail(SC_EINVAL, "gather waves %lld is not 4 or 8", (long long)v);
            p->gather_waves = (int)v;
            return SC_OK;
        case SC_PARAM_GATHER_MMA:
            if (v != SC_MMA_FP32 && v != SC_MMA_SPLIT16) return fail(SC_EINVAL, "gather product form %lld unknown", (long long)v);
            p->gather_mma = (int)v;
            return SC_OK;
        case SC_PARAM_RING_RPT: {
            if (v < 1 || v > 4) return fail(SC_EINVAL, "rings per lane %lld outside [1, 4]", (long long)v);
            if (p->prec == SC_MIXED) {
                p->rpt_mx = (int)v;
                p->ngroups_mx = sc_ring_groups(p->nring, (int)v);
            } else {
                p->rpt = (int)v;
                p->ngroups = sc_ring_groups(p->nring, (int)v);
            }
            return SC_OK;
        }
        case SC_PARAM_SKY_LMAX:
            if (v < p->lmax || v > 65535) return fail(SC_EINVAL, "sky lmax %lld below the plan's lmax %d", (long long)v, p->lmax);
            p->alm_lmax = (int)v;
            return SC_OK;
        case SC_PARAM_VALIDATE:
            if (v != 0 && v != 1) return fail(SC_EINVAL, "validate %lld is not 0 or 1", (long long)v);
            p->validate = (int)v;
            return SC_OK;
        case SC_PARAM_DETERMINISTIC:
            if (v != 0 && v != 1) return fail(SC_EINVAL, "deterministic %lld is not 0 or 1", (long long)v);
            if (v && !sc_scatter_binned_supported(p))
                return fail(SC_EINVAL, "the deterministic adjoint needs the binned FP32 scatter (W = 8, FP32 maps)");
            p->det_adjoint = (int)v;
            return SC_OK;
        default:
            return fail(SC_EINVAL, "unknown parameter %d", param);
    }
}

int sc_plan_get_param(const sc_plan *p, int param, int64_t *v) {
    if (!p || !v) return fail(SC_EINVAL, "NULL plan or output");
    switch (param) {
        case SC_PARAM_BIN_CHUNK: *v = p->bin_chunk; return SC_OK;
        case SC_PARAM_GATHER_WGS_PER_CU: *v = p->gather_wgs_per_cu; return SC_OK;
        case SC_PARAM_GATHER_WAVES: *v = p->gather_waves; return SC_OK;
        case SC_PARAM_GATHER_MMA: *v = p->gather_mma; return SC_OK;
        case SC_PARAM_RING_RPT: *v = p->prec == SC_MIXED ? p->rpt_mx : p->rpt; return SC_OK;
        case SC_PARAM_SKY_LMAX: *v = p->alm_lmax; return SC_OK;
        case SC_PARAM_VALIDATE: *v = p->validate; return SC_OK;
        case SC_PARAM_DETERMINISTIC: *v = p->det_adjoint; return SC_OK;
        default: return fail(SC_EINVAL, "unknown parameter %d", param);
    }
}

int sc_plan_enable_timing(sc_plan *p, int enable) {
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    p->timing = enable ? 1 : 0;
    return SC_OK;
}

int sc_plan_stage_times(sc_plan *p, double *ms, int64_t *launches, int nstage) {
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    double tot[SC_NSTAGE] = {};
    int64_t cnt[SC_NSTAGE] = {};
    for (int i = 0; i < p->tl_n; ++i) {
        TimedLaunch &t = p->tl[i];
        hipError_t e = hipEventSynchronize(t.b);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, t.a, t.b);
        if (e != hipSuccess) {
            p->tl_n = 0;
            return hip_fail(e, "stage timing events");
        }
        tot[t.stage] += f;
        cnt[t.stage] += 1;
    }
    p->tl_n = 0;
    for (int s = 0; s < nstage && s < SC_NSTAGE; ++s) {
        if (ms) ms[s] = tot[s];
        if (launches) launches[s] = cnt[s];
    }
    return SC_NSTAGE;
}

int64_t sc_debug_copy_stage(sc_plan *p, int which, void *dst, int64_t capacity) {
    if (!p || !dst) return fail(SC_EINVAL, "NULL plan or destination");
    if (!is_device_ptr(dst)) return fail(SC_EINVAL, "destination is not device memory");
    const void *src = nullptr;
    size_t bytes = 0;
    if (which == 0) {
        // complex128 in either storage
        src = p->F;
        const size_t n = (p->kmax + 1) * (2 * (size_t)p->lmax + 1) * p->nring;
        bytes = sizeof(double2) * n;
        if (p->mid32) {
            if ((int64_t)bytes > capacity)
                return fail(SC_EINVAL, "destination holds %lld bytes, need %zu", (long long)capacity, bytes);
            hipError_t e = sc_launch_widen((const float2 *)p->F, (double2 *)dst, n, p->stream);
            if (e != hipSuccess) return hip_fail(e, "stage copy");
            return (int64_t)bytes;
        }
    } else if (which == 1) {
        bytes = sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp;
        // column-tiled storage: reordered into (row, column, component)
        if ((int64_t)bytes > capacity)
            return fail(SC_EINVAL, "destination holds %lld bytes, need %zu", (long long)capacity, bytes);
        hipError_t e = sc_launch_maps_rowmajor(p, dst);
        if (e != hipSuccess) return hip_fail(e, "stage copy");
        return (int64_t)bytes;
    } else if (which == 2) {
        // the index field of each 32-byte sample record
        if (!p->bw.sorted.rec) return fail(SC_ESTATE, "no binning pass has run on this plan");
        const size_t nb = sizeof(int) * (size_t)p->bw.last_n;
        if ((int64_t)nb > capacity) return fail(SC_EINVAL, "destination holds %lld bytes, need %zu",
                                                (long long)capacity, nb);
        if (nb == 0) return 0;
        hipError_t e = hipMemcpy2DAsync(dst, sizeof(int), &p->bw.sorted.rec[0].idx, sizeof(BinRec), sizeof(int),
                                        (size_t)p->bw.last_n, hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "stage copy");
        return (int64_t)nb;
    } else {
        return fail(SC_EINVAL, "unknown stage %d", which);
    }
    if ((int64_t)bytes > capacity) return fail(SC_EINVAL, "destination holds %lld bytes, need %zu",
                                               (long long)capacity, bytes);
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "stage copy");
    return (int64_t)bytes;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of detectors: one shared sky, one plan (maps) per detector, one
// persistent gather launch over all detectors' work items; the whole sequence
// can be captured in a hipGraph and replayed.
struct sc_batch {
    int ndet, lmax_sky, prec;
    hipStream_t stream;
    std::vector<sc_plan *> plans;
    std::vector<sc_det_desc> dets;
    GatherDet *dets_dev;
    int *cursor;
    int max_ct;
    int wgs_per_cu;
    int waves;  // gather workgroup shape
    int mma;    // gather product form
    int warmed;
    hipGraph_t graph;
    hipGraphExec_t exec;
    const double *graph_alm;
    hipStream_t cap_stream;  // private stream for capture (the legacy null stream cannot be captured)
    hipEvent_t ev_stream;    // orders a new stream after the old one (sc_batch_set_stream)
    // Map synthesis and binning of the detectors run as SC_BATCH_CHAINS independent
    // chains: chain 0 on the batch's stream, the others on side streams forked from
    // it and joined before the gather; detectors are assigned by estimated work.
    hipStream_t side[3];
    hipEvent_t ev_fork, ev_join[3];
    std::vector<int> chain;  // chain of each detector
    int nchains;             // chains in use, 1 .. SC_BATCH_CHAINS (SC_PARAM_BATCH_CHAINS)
};

#define SC_BATCH_CHAINS 4

namespace {

void batch_drop_graph(sc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_alm = nullptr;
}

// Enqueue one full batch pass on stream s (no host synchronisation, capture-safe):
// fork the side chains from s, run each detector's map synthesis and binning on its
// chain, join, then the one gather launch over all detectors on s.  With `timed`
// (eager runs only, never under capture) and a plan's timing enabled, its launches
// are timed on its chain.
hipError_t batch_enqueue(sc_batch *b, const double *alm, hipStream_t s, bool timed) {
    auto tb = [timed](sc_plan *p, int stage) { return timed ? timing_begin(p, stage) : -1; };
    hipError_t e = hipEventRecord(b->ev_fork, s);
    for (int c = 0; c < SC_BATCH_CHAINS - 1 && e == hipSuccess; ++c) e = hipStreamWaitEvent(b->side[c], b->ev_fork, 0);
    for (int d = 0; d < b->ndet && e == hipSuccess; ++d) {
        sc_plan *p = b->plans[d];
        const sc_det_desc &D = b->dets[d];
        p->stream = b->chain[d] == 0 ? s : b->side[b->chain[d] - 1];
        int slot = tb(p, SC_STAGE_RING);
        e = p->prec == SC_MIXED ? sc_launch_ring_sums_mixed(p, alm, D.blm) : sc_launch_ring_sums(p, alm, D.blm);
        timing_end(p, slot);
        if (e == hipSuccess) {
            slot = tb(p, SC_STAGE_THETA);
            e = sc_launch_theta_upsample(p);
            timing_end(p, slot);
        }
        if (e == hipSuccess) {
            slot = tb(p, SC_STAGE_PHI);
            e = sc_launch_phi_synthesis(p);
            timing_end(p, slot);
        }
        if (e == hipSuccess) {
            slot = tb(p, SC_STAGE_BIN);
            e = D.n > 0 ? sc_launch_binning(p, D.ptg, D.n) : sc_launch_zero(p->bw.totals, 4 * sizeof(int), p->stream);
            timing_end(p, slot);
        }
    }
    for (int c = 0; c < SC_BATCH_CHAINS - 1; ++c) {
        // always join, so no side stream is left outside a capture
        const hipError_t e1 = hipEventRecord(b->ev_join[c], b->side[c]);
        const hipError_t e2 = hipStreamWaitEvent(s, b->ev_join[c], 0);
        if (e == hipSuccess) e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess) e = sc_launch_zero(b->cursor, sizeof(int), s);
    if (e == hipSuccess) {
        sc_plan *p0 = b->plans[0];
        p0->stream = s;
        const int slot = tb(p0, SC_STAGE_GATHER);  // the batch's one gather, on detector 0's record
        e = sc_launch_gather_batch(b->dets_dev, b->ndet, b->max_ct, b->cursor, b->wgs_per_cu, b->waves, b->mma, s);
        timing_end(p0, slot);
    }
    for (sc_plan *p : b->plans) p->stream = b->stream;
    return e;
}

double det_work(const sc_plan *p, int64_t n);

// Longest-processing-time assignment of the detectors to the batch's chains.
void batch_assign_chains(sc_batch *b) {
    const int ndet = b->ndet;
    std::vector<int> order(ndet);
    for (int d = 0; d < ndet; ++d) order[d] = d;
    std::vector<double> work(ndet);
    for (int d = 0; d < ndet; ++d) work[d] = det_work(b->plans[d], b->dets[d].n);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    double load[SC_BATCH_CHAINS] = {};
    b->chain.assign(ndet, 0);
    for (int d : order) {
        int best = 0;
        for (int c = 1; c < b->nchains; ++c)
            if (load[c] < load[best]) best = c;
        b->chain[d] = best;
        load[best] += work[d];
    }
}

// Estimated work of a detector (for the chain assignment): Wigner-d values of the
// ring sums plus multiply-adds of the gather.
double det_work(const sc_plan *p, int64_t n) {
    const double L = p->lmax + 1.0, K = p->kmax + 1.0;
    return K * L * L / 2.0 * p->nring * 6.0 + (double)n * (2.0 * p->kmax + 1.0) * p->W * p->W;
}

}  // namespace

extern "C" {

int sc_batch_destroy(sc_batch *b) {
    if (!b) return SC_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    for (int c = 0; c < SC_BATCH_CHAINS - 1; ++c)
        if (b->side[c]) {
            const hipError_t es = hipStreamSynchronize(b->side[c]);
            if (e == hipSuccess) e = es;
        }
    batch_drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ev_stream) (void)hipEventDestroy(b->ev_stream);
    for (int c = 0; c < SC_BATCH_CHAINS - 1; ++c) {
        if (b->side[c]) (void)hipStreamDestroy(b->side[c]);
        if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (sc_plan *p : b->plans) sc_plan_destroy(p);
    if (b->dets_dev) (void)hipFree(b->dets_dev);
    if (b->cursor) (void)hipFree(b->cursor);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize in sc_batch_destroy");
    return SC_OK;
}

int sc_batch_create(sc_batch **out, const sc_det_desc *dets, int ndet, int lmax_sky, int precision, void *stream) {
    g_msg[0] = 0;
    if (!out) return fail(SC_EINVAL, "batch output pointer is NULL");
    *out = nullptr;
    if (!dets || ndet < 1 || ndet > SC_MAX_DET) return fail(SC_EINVAL, "ndet = %d outside [1, %d]", ndet, SC_MAX_DET);
    if (precision != SC_F64MAPS_F32GATHER && precision != SC_MIXED)
        return fail(SC_EINVAL, "batches need FP32 maps (precision %d)", precision);
    for (int d = 0; d < ndet; ++d) {
        const sc_det_desc &D = dets[d];
        if (D.lmax < 0 || D.lmax > lmax_sky || D.kmax < 0 || D.kmax > D.lmax)
            return fail(SC_EINVAL, "detector %d: lmax %d / kmax %d invalid for sky lmax %d", d, D.lmax, D.kmax, lmax_sky);
        if (D.n < 0 || D.n > BIN_PASS_MAX)
            return fail(SC_EINVAL, "detector %d: n = %lld outside [0, %d]", d, (long long)D.n, BIN_PASS_MAX);
        if (!is_device_ptr(D.blm) || (D.n > 0 && (!is_device_ptr(D.ptg) || !is_device_ptr(D.tod))))
            return fail(SC_EINVAL, "detector %d: blm/ptg/tod is not device memory", d);
    }
    sc_batch *b = new (std::nothrow) sc_batch();
    if (!b) return fail(SC_ENOMEM, "host allocation failed");
    b->ndet = ndet;
    b->lmax_sky = lmax_sky;
    b->prec = precision;
    b->waves = 4;
    b->mma = SC_MMA_SPLIT16;
    b->stream = (hipStream_t)stream;
    b->dets.assign(dets, dets + ndet);
    std::vector<GatherDet> gd(ndet);
    for (int d = 0; d < ndet; ++d) {
        sc_plan *p = nullptr;
        int rc = sc_plan_create(&p, dets[d].lmax, dets[d].kmax, precision, 8, stream);
        if (!rc) {
            b->plans.push_back(p);
            p->alm_lmax = lmax_sky;
            rc = ensure_bin_work(p, dets[d].n > 0 ? dets[d].n : 1);
            p->bin_fixed = 1;
        }
        if (rc) {
            sc_batch_destroy(b);
            return rc;
        }
        gd[d] = sc_gather_det(p, dets[d].tod);
        const int ct = (p->ncomp + 15) / 16;
        if (ct > b->max_ct) b->max_ct = ct;
    }
    size_t tot = 0;
    int rc = alloc((void **)&b->dets_dev, sizeof(GatherDet) * ndet, &tot);
    if (!rc) rc = alloc((void **)&b->cursor, sizeof(int), &tot);
    if (rc) {
        sc_batch_destroy(b);
        return rc;
    }
    {
        // side streams (default priority) and events of the synthesis chains
        hipError_t es = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        for (int c = 0; c < SC_BATCH_CHAINS - 1 && es == hipSuccess; ++c) {
            es = hipStreamCreateWithFlags(&b->side[c], hipStreamNonBlocking);
            if (es == hipSuccess) es = hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming);
        }
        if (es != hipSuccess) {
            sc_batch_destroy(b);
            return hip_fail(es, "batch side streams");
        }
        b->nchains = SC_BATCH_CHAINS;
        batch_assign_chains(b);
    }
    hipError_t e = hipMemcpyAsync(b->dets_dev, gd.data(), sizeof(GatherDet) * ndet, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        sc_batch_destroy(b);
        return hip_fail(e, "batch descriptor upload");
    }
    *out = b;
    return SC_OK;
}

int sc_batch_set_param(sc_batch *b, int det, int param, int64_t value) {
    if (!b) return fail(SC_EINVAL, "batch is NULL");
    if (param == SC_PARAM_GATHER_WGS_PER_CU) {
        if (value < 0 || value > 16) return fail(SC_EINVAL, "workgroups per CU outside [0, 16]");
        b->wgs_per_cu = (int)value;
        batch_drop_graph(b);
        return SC_OK;
    }
    if (param == SC_PARAM_BATCH_CHAINS) {
        if (value < 1 || value > SC_BATCH_CHAINS)
            return fail(SC_EINVAL, "synthesis chains %lld outside [1, %d]", (long long)value, SC_BATCH_CHAINS);
        b->nchains = (int)value;
        batch_assign_chains(b);
        batch_drop_graph(b);
        return SC_OK;
    }
    if (param == SC_PARAM_GATHER_WAVES) {
        if (value != 4 && value != 8) return fail(SC_EINVAL, "gather waves %lld is not 4 or 8", (long long)value);
        b->waves = (int)value;
        batch_drop_graph(b);
        return SC_OK;
    }
    if (param == SC_PARAM_GATHER_MMA) {
        if (value != SC_MMA_FP32 && value != SC_MMA_SPLIT16)
            return fail(SC_EINVAL, "gather product form %lld unknown", (long long)value);
        b->mma = (int)value;
        batch_drop_graph(b);
        return SC_OK;
    }
    if (param == SC_PARAM_SKY_LMAX) return fail(SC_EINVAL, "the sky lmax of a batch is fixed at creation");
    if (det < -1 || det >= b->ndet) return fail(SC_EINVAL, "detector %d outside [-1, %d)", det, b->ndet);
    for (int d = 0; d < b->ndet; ++d) {
        if (det >= 0 && d != det) continue;
        int rc = sc_plan_set_param(b->plans[d], param, value);
        if (rc) return rc;
    }
    batch_drop_graph(b);
    return SC_OK;
}

int sc_batch_get_param(const sc_batch *b, int det, int param, int64_t *value) {
    if (!b || !value) return fail(SC_EINVAL, "NULL batch or output");
    if (param == SC_PARAM_GATHER_WGS_PER_CU) {
        *value = b->wgs_per_cu;
        return SC_OK;
    }
    if (param == SC_PARAM_GATHER_WAVES) {
        *value = b->waves;
        return SC_OK;
    }
    if (param == SC_PARAM_BATCH_CHAINS) {
        *value = b->nchains;
        return SC_OK;
    }
    if (param == SC_PARAM_GATHER_MMA) {
        *value = b->mma;
        return SC_OK;
    }
    if (det < 0 || det >= b->ndet) return fail(SC_EINVAL, "detector %d outside [0, %d)", det, b->ndet);
    return sc_plan_get_param(b->plans[det], param, value);
}

int sc_batch_run(sc_batch *b, const double *alm_sky, int use_graph) {
    g_msg[0] = 0;
    if (!b) return fail(SC_EINVAL, "batch is NULL");
    if (!is_device_ptr(alm_sky) || ((uintptr_t)alm_sky & 15)) return fail(SC_EINVAL, "alm_sky is not aligned device memory");
    hipError_t e = hipSuccess;
    if (!use_graph) {
        e = batch_enqueue(b, alm_sky, b->stream, true);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        return SC_OK;
    }
    if (b->exec && b->graph_alm == alm_sky) {
        e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return SC_OK;
    }
    if (!b->warmed) {
        // one eager pass first: kernel attributes and launch shapes get cached
        // outside the capture
        e = batch_enqueue(b, alm_sky, b->stream, true);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        b->warmed = 1;
    }
    batch_drop_graph(b);
    if (!b->cap_stream) {
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            b->cap_stream = nullptr;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
    }
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t e2 = batch_enqueue(b, alm_sky, b->cap_stream, false);
    e = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (e2 != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(e2, "batch capture");
    }
    if (e != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        batch_drop_graph(b);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph_alm = alm_sky;
    e = hipGraphLaunch(b->exec, b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SC_OK;
}

int sc_batch_set_stream(sc_batch *b, void *stream) {
    g_msg[0] = 0;
    if (!b) return fail(SC_EINVAL, "batch is NULL");
    hipStream_t next = (hipStream_t)stream;
    if (next == b->stream) return SC_OK;
    hipError_t e = hipSuccess;
    if (!b->ev_stream) e = hipEventCreateWithFlags(&b->ev_stream, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->ev_stream, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, b->ev_stream, 0);
    if (e != hipSuccess) return hip_fail(e, "ordering the new stream after the batch's stream");
    b->stream = next;
    for (sc_plan *p : b->plans) p->stream = next;
    return SC_OK;
}

int sc_batch_plan(sc_batch *b, int det, sc_plan **plan) {
    if (!b || !plan || det < 0 || det >= b->ndet) return fail(SC_EINVAL, "bad batch, detector or output");
    *plan = b->plans[det];
    return SC_OK;
}

}  // extern "C"
