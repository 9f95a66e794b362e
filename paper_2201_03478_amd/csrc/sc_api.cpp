// sc_api.cpp -- C ABI of libsidelobe: argument validation, plan geometry and
// workspace, and the order of kernel launches.  No arithmetic of the method
// happens on the host: every stage runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

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

bool factor_fft(int n, FftPlan *P) {
    P->n = n;
    P->nst = 0;
    int m = n;
    while (m % 4 == 0 && P->nst < SC_MAX_RADICES) { P->r[P->nst++] = 4; m /= 4; }
    while (m % 2 == 0 && P->nst < SC_MAX_RADICES) { P->r[P->nst++] = 2; m /= 2; }
    while (m % 3 == 0 && P->nst < SC_MAX_RADICES) { P->r[P->nst++] = 3; m /= 3; }
    while (m % 5 == 0 && P->nst < SC_MAX_RADICES) { P->r[P->nst++] = 5; m /= 5; }
    return m == 1 && n <= 16 * 512;  // longest transform the LDS kernels handle
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

void free_bin_work(BinWork &w) {
    void *bufs[] = {w.count, w.offs, w.sums, w.totals, w.key, w.rank, w.sorted.fu, w.sorted.fv,
                    w.sorted.psi, w.sorted.idx, w.items};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    std::memset(&w, 0, sizeof(w));
}

int alloc(void **dst, size_t bytes, size_t *total);

// Binning workspace for passes of up to `need` samples (grown on demand).
int ensure_bin_work(sc_plan *p, int64_t need) {
    BinWork &w = p->bw;
    if (w.cap >= need) return SC_OK;
    // buffers are in use by earlier work on the stream until it completes
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail(SC_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    p->ws_bytes -= w.bytes;
    free_bin_work(w);
    const BinGeom g = sc_bin_geom(p);
    const int64_t nkeys = (int64_t)g.nkr * g.nkc;
    const int64_t nblk = (nkeys + 4095) / 4096;
    size_t tot = 0;
    int rc = SC_OK;
    rc = rc ? rc : alloc((void **)&w.count, sizeof(int) * nkeys, &tot);
    rc = rc ? rc : alloc((void **)&w.offs, sizeof(int2) * nkeys, &tot);
    rc = rc ? rc : alloc((void **)&w.sums, sizeof(int2) * nblk, &tot);
    rc = rc ? rc : alloc((void **)&w.totals, sizeof(int) * 4, &tot);
    rc = rc ? rc : alloc((void **)&w.key, sizeof(int) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.rank, sizeof(int) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.sorted.fu, sizeof(double) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.sorted.fv, sizeof(double) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.sorted.psi, sizeof(double) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.sorted.idx, sizeof(int) * need, &tot);
    rc = rc ? rc : alloc((void **)&w.items, sizeof(int4) * need, &tot);
    if (rc) {
        free_bin_work(w);
        return rc;
    }
    w.cap = need;
    w.nkeys = nkeys;
    w.bytes = tot;
    p->ws_bytes += tot;
    return SC_OK;
}

void free_plan_buffers(sc_plan *p) {
    free_bin_work(p->bw);
    if (p->gmaps) (void)hipFree(p->gmaps);
    if (p->GA) (void)hipFree(p->GA);
    p->gmaps = nullptr;
    p->GA = nullptr;
    for (int i = 0; i < p->tl_cap; ++i) {
        if (p->tl[i].a) (void)hipEventDestroy(p->tl[i].a);
        if (p->tl[i].b) (void)hipEventDestroy(p->tl[i].b);
    }
    std::free(p->tl);
    p->tl = nullptr;
    p->tl_cap = p->tl_n = 0;
    void *bufs[] = {p->F, p->G, p->maps, p->sbin_m, p->sbin_e, p->tw2, p->tw2os, p->twphi,
                    p->phase, p->dphi, p->glx, p->glw};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

int alloc(void **dst, size_t bytes, size_t *total) {
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    *total += bytes;
    return SC_OK;
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
    p->nphi = next_smooth(2 * (2 * lmax + 1), false);
    if (p->nphi < 2 * W) p->nphi = next_smooth(2 * W, false);
    p->rows = p->n2os / 2 + W;
    p->cols = p->nphi + W - 1;
    p->ncomp = 2 * kmax + 1;
    p->ncp = (p->ncomp + 3) & ~3;
    p->nq = 128;
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
    if (!factor_fft(p->n2, &p->p2) || !factor_fft(p->n2os, &p->p2os) || !factor_fft(p->nphi, &p->pphi)) {
        delete p;
        return fail(SC_EINVAL, "lmax = %d needs transforms longer than 8192 points (not supported)", lmax);
    }

    const size_t nm = 2 * (size_t)lmax + 1;
    size_t tot = 0;
    int rc = SC_OK;
    rc = rc ? rc : alloc((void **)&p->F, sizeof(double2) * (kmax + 1) * nm * p->nring, &tot);
    rc = rc ? rc : alloc((void **)&p->G, sizeof(double2) * (kmax + 1) * (size_t)p->rows * nm, &tot);
    rc = rc ? rc : alloc(&p->maps, sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp, &tot);
    rc = rc ? rc : alloc((void **)&p->sbin_m, sizeof(double) * (lmax + 1) * (kmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->sbin_e, sizeof(int) * (lmax + 1) * (kmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->tw2, sizeof(double2) * p->n2, &tot);
    rc = rc ? rc : alloc((void **)&p->tw2os, sizeof(double2) * p->n2os, &tot);
    rc = rc ? rc : alloc((void **)&p->twphi, sizeof(double2) * p->nphi, &tot);
    rc = rc ? rc : alloc((void **)&p->phase, sizeof(double2) * nm, &tot);
    rc = rc ? rc : alloc((void **)&p->dphi, sizeof(double) * (lmax + 1), &tot);
    rc = rc ? rc : alloc((void **)&p->glx, sizeof(double) * p->nq, &tot);
    rc = rc ? rc : alloc((void **)&p->glw, sizeof(double) * p->nq, &tot);
    if (rc) {
        free_plan_buffers(p);
        delete p;
        return rc;
    }
    p->ws_bytes = tot;
    // padding components stay zero for the plan's lifetime
    hipError_t e = hipMemsetAsync(p->maps, 0, sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp, p->stream);
    if (e == hipSuccess) e = sc_launch_tables(p);
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
    free_plan_buffers(p);
    delete p;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize in sc_plan_destroy");
    return SC_OK;
}

int sc_plan_set_stream(sc_plan *p, void *stream) {
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    p->stream = (hipStream_t)stream;
    return SC_OK;
}

int sc_plan_info(const sc_plan *p, int64_t *out, int nout) {
    if (!p || (nout > 0 && !out)) return fail(SC_EINVAL, "NULL plan or output");
    const int64_t v[] = {p->lmax, p->kmax, p->prec, p->W, p->nring, p->n2, p->n2os, p->nphi,
                         p->rows, p->cols, p->ncomp, p->ncp, (int64_t)p->ws_bytes};
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
    return SC_OK;
}

int sc_interpolate(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (n == 0) return SC_OK;
    if (!p->have_maps) return fail(SC_ESTATE, "sc_interpolate before sc_set_sky_beam");
    if (!is_device_ptr(ptg)) return fail(SC_EINVAL, "ptg is not device memory");
    if (!is_device_ptr(tod)) return fail(SC_EINVAL, "tod is not device memory");
    if (((uintptr_t)ptg & 7) || ((uintptr_t)tod & (p->prec == SC_FP64 ? 7 : 3)))
        return fail(SC_EINVAL, "ptg/tod misaligned");
    if (p->gather_direct || !sc_gather_binned_supported(p)) {
        int slot = timing_begin(p, SC_STAGE_GATHER);
        hipError_t e = sc_launch_gather(p, ptg, n, tod);
        timing_end(p, slot);
        if (e != hipSuccess) return hip_fail(e, "gather launch");
        return SC_OK;
    }
    const int64_t pass = n < p->bin_pass_max ? n : p->bin_pass_max;
    int rc = ensure_bin_work(p, pass);
    if (rc) return rc;
    const size_t esz = p->prec == SC_FP64 ? 8 : 4;
    for (int64_t off = 0; off < n; off += pass) {
        const int64_t cnt = n - off < pass ? n - off : pass;
        int slot = timing_begin(p, SC_STAGE_BIN);
        hipError_t e = sc_launch_binning(p, ptg + 3 * off, cnt);
        timing_end(p, slot);
        if (e != hipSuccess) return hip_fail(e, "binning launch");
        slot = timing_begin(p, SC_STAGE_GATHER);
        e = sc_launch_gather_binned(p, (char *)tod + esz * off);
        timing_end(p, slot);
        if (e != hipSuccess) return hip_fail(e, "binned gather launch");
    }
    return SC_OK;
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
        p->stream = (hipStream_t)stream;
    }
    int rc = sc_set_sky_beam(p, alm, blm);
    if (rc) return rc;
    return sc_interpolate(p, ptg, n, tod);
}

int sc_convolve_adjoint(sc_plan *p, const double *blm, const double *ptg, const void *tod_grad, int64_t n,
                        double *alm_grad) {
    g_msg[0] = 0;
    if (!p) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (!is_device_ptr(blm)) return fail(SC_EINVAL, "blm is not device memory");
    if (!is_device_ptr(alm_grad)) return fail(SC_EINVAL, "alm_grad is not device memory");
    if (n > 0 && (!is_device_ptr(ptg) || !is_device_ptr(tod_grad)))
        return fail(SC_EINVAL, "ptg/tod_grad is not device memory");
    if (((uintptr_t)blm & 15) || ((uintptr_t)alm_grad & 15)) return fail(SC_EINVAL, "blm/alm_grad not 16-byte aligned");
    if (n > 0 && (((uintptr_t)ptg & 7) || ((uintptr_t)tod_grad & (p->prec == SC_FP64 ? 7 : 3))))
        return fail(SC_EINVAL, "ptg/tod_grad misaligned");
    const size_t map_bytes = sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp;
    const size_t nalm = (size_t)(p->lmax + 1) * (p->lmax + 2) / 2;
    if (!p->gmaps) {
        size_t tot = 0;
        int rc = alloc(&p->gmaps, map_bytes, &tot);
        if (!rc) rc = alloc((void **)&p->GA, sizeof(double2) * (p->kmax + 1) * nalm, &tot);
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
            const size_t esz = p->prec == SC_FP64 ? 8 : 4;
            for (int64_t off = 0; off < n; off += pass) {
                const int64_t cnt = n - off < pass ? n - off : pass;
                slot = timing_begin(p, SC_STAGE_BIN);
                e = sc_launch_binning(p, ptg + 3 * off, cnt);
                timing_end(p, slot);
                if (e != hipSuccess) return hip_fail(e, "binning launch");
                slot = timing_begin(p, SC_STAGE_SCATTER);
                e = sc_launch_scatter_binned(p, (const char *)tod_grad + esz * off, p->gmaps);
                timing_end(p, slot);
                if (e != hipSuccess) return hip_fail(e, "binned scatter launch");
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
    slot = timing_begin(p, SC_STAGE_ADJ_RING);
    e = sc_launch_ring_sums_adjoint(p, blm, alm_grad);
    timing_end(p, slot);
    if (e != hipSuccess) return hip_fail(e, "adjoint ring-sum launch");
    return SC_OK;
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
        src = p->F;
        bytes = sizeof(double2) * (p->kmax + 1) * (2 * (size_t)p->lmax + 1) * p->nring;
    } else if (which == 1) {
        src = p->maps;
        bytes = sc_map_elem_bytes(p) * (size_t)p->rows * p->cols * p->ncp;
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
