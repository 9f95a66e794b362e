// sc_noalloc.cpp -- interpolation that allocates nothing (sc_interpolate_noalloc).
//
// Callers that cannot allocate device memory (code under graph capture, tight
// serving loops) get the binned interpolation of sc_interpolate with its binning
// workspace (anchor counts and offsets, scan sums, totals and the work-queue
// cursor, per-sample keys and ranks, sorted sample records, work items) in one
// fixed device array per GPU instead of plan workspace.  The array's name is a
// host-side stand-in: host code passes kernels the device address that
// hipGetSymbolAddress returned for the current device (looked up once per device,
// on the first call there).  Every call on a GPU shares that GPU's array, so calls
// that overlap on one GPU (two streams, two plans, two threads) race.  Everything
// that must start at zero (anchor counts, the work cursor) is cleared by the
// binning kernels of each pass; no memset is used.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "sc_common.h"

#define SC_NOALLOC_SCRATCH_BYTES (256u << 20)
static __device__ __align__(256) unsigned char scratch[SC_NOALLOC_SCRATCH_BYTES];

namespace {

struct ScratchTable {
    std::mutex mu;
    void *ptr[64] = {};
};
ScratchTable &scratch_table() {
    static ScratchTable *t = new ScratchTable();
    return *t;
}

// Device address of the current device's scratch array (looked up on first use).
int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sc_hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return sc_error(SC_EINVAL, "device %d outside the 64 the scratch table holds", dev);
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return sc_hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return sc_error(SC_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        t.ptr[dev] = ptr;
    }
    *out = t.ptr[dev];
    return SC_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// The binning workspace carved out of `bytes` bytes at `base`: the per-anchor tables
// (12 bytes per anchor), then as many samples per pass as the rest holds (56 bytes
// each, a multiple of 256).  Returns the pass size, or 0 if fewer than
// kMinPass samples would fit beside the anchor tables.
constexpr int64_t kMinPass = 4096;
int64_t carve_bin_work(const sc_plan *p, unsigned char *base, size_t bytes, BinWork *w) {
    const BinGeom g = sc_bin_geom(p);
    const int64_t nkeys = (int64_t)g.nkr * g.nkc;
    const int64_t nblk = (nkeys + 4095) / 4096;
    std::memset(w, 0, sizeof(*w));
    size_t off = 0;
    w->count = (int *)(base + off);
    off += align_up(sizeof(int) * nkeys);
    w->offs = (int2 *)(base + off);
    off += align_up(sizeof(int2) * nkeys);
    w->sums = (int2 *)(base + off);
    off += align_up(sizeof(int2) * nblk);
    w->totals = (int *)(base + off);
    off += align_up(sizeof(int) * 4);
    const size_t per = 2 * sizeof(int) + sizeof(BinRec) + sizeof(int4);
    if (off + 4 * 256 + per * kMinPass > bytes) return 0;
    const int64_t cap = (int64_t)((bytes - off - 4 * 256) / per) & ~(int64_t)255;
    w->key = (int *)(base + off);
    off += align_up(sizeof(int) * cap);
    w->rank = (int *)(base + off);
    off += align_up(sizeof(int) * cap);
    w->sorted.rec = (BinRec *)(base + off);
    off += align_up(sizeof(BinRec) * cap);
    w->items = (int4 *)(base + off);
    off += align_up(sizeof(int4) * cap);
    if (off > bytes) return 0;
    w->cap = cap;
    w->nkeys = nkeys;
    return cap;
}

}  // namespace

extern "C" int sc_interpolate_noalloc(sc_plan *p, const double *ptg, int64_t n, void *tod) {
    sc_clear_error();
    if (!p) return sc_error(SC_EINVAL, "plan is NULL");
    if (n < 0) return sc_error(SC_EINVAL, "n = %lld < 0", (long long)n);
    if (n == 0) return SC_OK;
    if (!p->have_maps) return sc_error(SC_ESTATE, "sc_interpolate_noalloc before sc_set_sky_beam");
    int rc = sc_check_interp_args(p, ptg, tod);
    if (rc) return rc;
    if (!sc_uses_binning(p)) {  // the per-sample gather needs no workspace
        const hipError_t e = sc_launch_gather(p, ptg, n, tod);
        return e != hipSuccess ? sc_hip_error(e, "gather launch") : SC_OK;
    }
    void *base = nullptr;
    rc = scratch_ptr(&base);
    if (rc) return rc;
    BinWork view;
    const int64_t cap = carve_bin_work(p, (unsigned char *)base, SC_NOALLOC_SCRATCH_BYTES, &view);
    if (cap == 0) {
        const BinGeom g = sc_bin_geom(p);
        const long long nk = (long long)g.nkr * g.nkc;
        return sc_error(SC_EINVAL,
                        "sc_interpolate_noalloc: lmax %d has %lld interpolation anchors (%lld bytes of tables); "
                        "the %u-byte scratch must also hold %lld samples",
                        p->lmax, nk, 12 * nk, (unsigned)SC_NOALLOC_SCRATCH_BYTES, (long long)kMinPass);
    }
    const int64_t pass = cap < p->bin_pass_max ? cap : p->bin_pass_max;
    const size_t esz = p->prec == SC_FP64 ? 8 : 4;
    const BinWork own = p->bw;
    p->bw = view;  // the launchers take their buffers from p->bw
    hipError_t e = hipSuccess;
    for (int64_t off = 0; off < n && e == hipSuccess; off += pass) {
        const int64_t cnt = n - off < pass ? n - off : pass;
        e = sc_launch_binning(p, ptg + 3 * off, cnt);
        if (e == hipSuccess) e = sc_launch_gather_binned(p, (char *)tod + esz * off);
    }
    p->bw = own;
    return e != hipSuccess ? sc_hip_error(e, "no-allocation interpolation launch") : SC_OK;
}
