/*
 * sidelobe.h -- C ABI of the MI355X (gfx950) spin-harmonic total convolution.
 *
 * The library evaluates the total convolution of a sky and a beam
 * (Galloway et al. 2022, "BeyondPlanck VIII", Sec. 2.1, Eqs. 1-2):
 *
 *   c(theta, phi, psi) = sum_{l,m,k} a_lm conj(b_lk) [D^l_mk(phi, theta, psi)]*
 *                      = sum_{l,m,k} a_lm conj(b_lk) e^{i m phi} d^l_mk(theta) e^{i k psi},
 *
 * for a real sky a_lm (l <= lmax) and a real beam b_lk truncated at |k| <= kmax,
 * by the two-step method of Sec. 2.1: one spin-k transform per beam order k
 * (Eqs. 7 and 9) gives the component maps T_k(theta, phi); the +-k pairs
 * combine as 2[cos k psi Re T_k - sin k psi Im T_k] (Eq. 8).  Here the maps
 * are synthesised on an oversampled equiangular grid (Wigner-d recursion over
 * l, per-m ring contraction, ring FFTs) and the signal is interpolated at each
 * pointing with an exponential-of-semicircle kernel, the k-sum done per sample
 * (the finite-resolution cube plus interpolation described at the end of
 * Sec. 2.1).
 *
 * Conventions
 *   D^l_mk(a, b, g) = e^{-i m a} d^l_mk(b) e^{-i k g}, d the standard
 *   (Condon-Shortley compatible) small d-matrix; the beam is defined pointing
 *   at the north pole and is placed by the active rotation
 *   R = R_z(phi) R_y(theta) R_z(psi).
 *
 * Layouts (all caller buffers are DEVICE memory, owned by the caller)
 *   alm   complex128 (re, im interleaved), m-major triangular:
 *         index(l, m) = m (2 lmax + 1 - m) / 2 + l,  0 <= m <= l <= lmax.
 *         Im(a_l0) is ignored (real sky).
 *   blm   complex128, same scheme with m -> k and k <= kmax:
 *         index(l, k) = k (2 lmax + 1 - k) / 2 + l,  0 <= k <= min(l, kmax);
 *         (kmax + 1)(lmax + 1) - kmax (kmax + 1)/2 entries.  Im(b_l0) ignored.
 *         Negative orders follow from the real-field symmetry (Eq. 6).
 *   ptg   float64 [n][3] = (theta, phi, psi) in radians, theta in [0, pi];
 *         phi and psi are reduced modulo 2 pi.
 *   tod   float64 [n] for SC_FP64 plans, float32 [n] otherwise.
 *
 * Streams, ordering, threads
 *   Every call enqueues work on the plan's HIP stream and returns without
 *   synchronising the device.  Changing a plan's stream (sc_plan_set_stream,
 *   or a cached one-shot plan called with another stream) makes the new
 *   stream wait for everything already queued on the old one, so the plan's
 *   workspace is never used by two streams at once.  A plan is not
 *   thread-safe: do not call it from two host threads at once.  Inputs must
 *   stay valid until the stream reaches the work.  Workspace that grows on
 *   demand (the pointing-binning buffers, the psi cube) is allocated and
 *   released in stream order (hipMallocAsync / hipFreeAsync), so no call
 *   after sc_plan_create waits for the device, except sc_plan_destroy,
 *   sc_plan_stage_times and sc_batch_create/destroy, which say so.
 *
 * Errors
 *   Every entry point returns SC_OK or a negative code and never aborts or
 *   throws.  sc_last_error() returns a message for the calling thread's last
 *   failure.  Invalid arguments (negative sizes, kmax > lmax, null pointers,
 *   host pointers where device memory is required, misaligned buffers) give
 *   SC_EINVAL without touching the device; allocation failure gives
 *   SC_ENOMEM; a failed HIP call gives SC_EHIP; calls in the wrong order
 *   (interpolating before maps exist) give SC_ESTATE.  n = 0 is a valid no-op.
 */
#ifndef SIDELOBE_H
#define SIDELOBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_plan sc_plan;

/* Largest supported band limit. */
#define SC_LMAX_MAX 8192

enum sc_status {
    SC_OK = 0,
    SC_EINVAL = -1,
    SC_ENOMEM = -2,
    SC_EHIP = -3,
    SC_ESTATE = -4
};

/* Arithmetic of a plan. */
enum sc_precision {
    /* FP64 recursion, transforms, maps, interpolation and k-sum; float64 TOD. */
    SC_FP64 = 0,
    /* FP64 recursion and transforms; maps stored in FP32; FP32 interpolation
       and k-sum (pointing reduction and psi reduction stay FP64); float32 TOD. */
    SC_F64MAPS_F32GATHER = 1,
    /* Precision variant: the FP64 Wigner-d recursion of SC_F64MAPS_F32GATHER,
       with the ring contraction on the matrix cores (d values and coefficient
       products rounded to FP32, FP32 products, FP32 accumulation over 64
       steps, then FP64 sums); FP64 transforms; FP32 maps, interpolation and
       k-sum; float32 TOD. */
    SC_MIXED = 2
};

/*
 * Create a plan for one (lmax, kmax, precision).
 *   lmax          0 <= lmax <= SC_LMAX_MAX (8192), band limit of sky and beam.
 *                 The theta and phi transforms (about 2 lmax and 4 lmax
 *                 points) run in one workgroup's LDS up to 9216 points; above
 *                 that (lmax > 2303) each runs as several LDS transforms through
 *                 an extra (kmax + 1)(2 lmax + 1)^2 complex128 plan buffer.
 *                 Larger lmax: SC_EINVAL.
 *   kmax          0 <= kmax <= min(lmax, 127), beam azimuthal truncation
 *                 (kmax = 0 is the axisymmetric case, a spin-0 transform only;
 *                 Sec. 2.1).
 *   precision     an sc_precision value.
 *   kernel_width  interpolation kernel width W in grid cells (even, 4..16), or
 *                 0 for the default (8 for SC_F64MAPS_F32GATHER, 14 for SC_FP64).
 *   stream        hipStream_t to enqueue on (NULL = the null stream).
 * The plan allocates all of its device workspace here (maps, transform
 * buffers, tables) and fills its constant tables on the stream.
 */
int sc_plan_create(sc_plan **plan, int lmax, int kmax, int precision, int kernel_width, void *stream);

/* Release a plan and its workspace (synchronises its stream first). NULL is a no-op. */
int sc_plan_destroy(sc_plan *plan);

/* Change the stream a plan enqueues on.  The new stream first waits (an event,
   no host wait) for all work queued on the old one. */
int sc_plan_set_stream(sc_plan *plan, void *stream);

/*
 * Plan geometry, written to out[0 .. nout-1] in this order:
 *   0 lmax, 1 kmax, 2 precision, 3 W, 4 n_rings (theta rings of the
 *   recursion), 5 n_fft_theta (2 n_rings), 6 n_theta_fine (oversampled
 *   full-circle theta grid), 7 n_phi (oversampled phi grid), 8 map_rows,
 *   9 map_cols, 10 n_comp (2 kmax + 2: a cos k psi, sin k psi
 *   pair per k, the sin 0 psi slot zero), 11 n_comp_padded,
 *   12 workspace bytes, 13 bytes per complex value of the forward path's ring
 *   sums and upsampled spectra (16; 8 in the FP32-map forms up to lmax 2303,
 *   whose transforms fit one workgroup: computed in FP64, stored as complex64).
 * Returns the number of values available (14).
 */
int sc_plan_info(const sc_plan *plan, int64_t *out, int nout);

/*
 * Synthesise the component maps for a sky and a beam (the spin transforms of
 * Eq. 9, one per k = 0..kmax; Eq. 7 reordered with the k sum outside).
 * alm, blm: device complex128 arrays in the layouts above.  The maps stay
 * resident in the plan until the next call.
 */
int sc_set_sky_beam(sc_plan *plan, const double *alm, const double *blm);

/*
 * Evaluate the convolution at n pointings from the plan's maps: interpolate
 * every component at (theta, phi) and sum the cos k psi / sin k psi terms
 * (Eq. 8).  ptg: device float64 [n][3]; tod: device float64/float32 [n].
 */
int sc_interpolate(sc_plan *plan, const double *ptg, int64_t n, void *tod);

/*
 * sc_interpolate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * result from the same kernels, with the binning workspace in a fixed 256 MiB
 * device array that the library holds on each GPU it runs on until the process
 * ends, instead of plan workspace.  Samples are binned in passes of what the
 * array holds beside the plan's anchor tables (12 bytes per interpolation
 * anchor, 56 bytes per sample), so n is not limited; a grid whose anchor
 * tables leave no room for 4096 samples (lmax above about 1400) returns
 * SC_EINVAL.  Calls no hipMalloc, hipFree or other allocating routine (the
 * array's device address is looked up on the first call on each device).
 * Every call on one GPU shares that GPU's array: calls that overlap on a GPU
 * (other streams, plans or threads) race, so the caller orders them.  Same
 * arguments, layouts, stream and errors as sc_interpolate.
 */
int sc_interpolate_noalloc(sc_plan *plan, const double *ptg, int64_t n, void *tod);

/*
 * The second step of the two-step algorithm (Sec. 2.1): the Fourier series over
 * k of the plan's current component maps, evaluated on a grid of npsi points in
 * psi at every (theta, phi) grid point and divided by the interpolation
 * kernel's transform along psi, giving the real cube c(theta, phi, psi).
 * npsi = 0 picks the smallest product of 2, 3 and 5 >= max(2 (2 kmax + 1), 2 W);
 * an explicit npsi must be such a product in [that bound, 512], else
 * SC_EINVAL.  The cube (rows x cols x (npsi + W - 1 rounded up to 4) values of
 * the map type, about 2 npsi / (2 kmax + 2) times the maps) is allocated by the
 * plan on the first call or when npsi changes, and freed with the plan; a call
 * before sc_set_sky_beam returns SC_ESTATE.  A later sc_set_sky_beam or
 * sc_plan_convolve invalidates the cube.  Asynchronous on the plan's stream.
 */
int sc_plan_build_psi_cube(sc_plan *plan, int npsi);

/*
 * Evaluate the convolution at n pointings by interpolating the cube in theta,
 * phi and psi with the same kernel (W^3 cube values per sample).  It
 * approximates the same quantity as sc_interpolate, with the kernel's error
 * in psi added.  ptg: device float64 [n][3]; tod: device float64/float32 [n]
 * (the map type).  FP32 plans with W = 8 first bin the samples by stencil
 * anchor in the plan's binning workspace (as sc_interpolate does, in passes of
 * at most 2^27 samples); only the order in which samples are processed
 * changes, not their values.  Without a cube of the current maps: SC_ESTATE;
 * host memory or misaligned pointers: SC_EINVAL.  n = 0 is a no-op.
 */
int sc_interpolate_psi(sc_plan *plan, const double *ptg, int64_t n, void *tod);

/*
 * sc_set_sky_beam followed by sc_interpolate, as one call: the pointing binning
 * of the first pass (it needs only ptg) runs on a plan-owned side stream while
 * the maps are synthesised, and joins the plan's stream before the gather.
 * Same arguments, layouts and errors as the two calls; the side stream is
 * created on first use, waits for all work queued before the call, and holds
 * no work after the call's own gather.
 */
int sc_plan_convolve(sc_plan *plan, const double *alm, const double *blm, const double *ptg, int64_t n,
                     void *tod);

/*
 * One-shot convolve(alm, blm, lmax, kmax, pointings) -> tod: creates (or
 * reuses a cached) plan for (lmax, kmax, precision, default W) on the current
 * device, moves it to `stream` (ordered after its previous stream, as
 * sc_plan_set_stream does) and runs sc_plan_convolve on it.  Same layouts as
 * above.  Calls from several host threads are serialised.  Cached plans keep
 * their workspace until sc_convolve_release_cache.
 */
int sc_convolve(const double *alm, const double *blm, int lmax, int kmax,
                const double *ptg, int64_t n, void *tod, int precision, void *stream);

/* Destroy every plan cached by sc_convolve (waits for their streams). */
int sc_convolve_release_cache(void);

/*
 * Adjoint of the convolution with respect to the sky coefficients (the
 * transpose of every stage above: scatter of the TOD gradient onto gradient
 * maps, adjoint phi and theta transforms, adjoint Wigner-d ring sums).  For a
 * TOD gradient y it returns g_lm = dL/dRe(a_lm) + i dL/dIm(a_lm) of
 * L = sum_t y_t c_t, i.e. <y, A a> = Re sum_{l, m >= 0} conj(g_lm) a_lm;
 * g_l0 is real.  This is torch's complex-gradient convention.
 *   blm       device complex128, the beam the plan's maps were made with.
 *   ptg       device float64 [n][3].
 *   tod_grad  device float64 [n] (SC_FP64) or float32 [n].
 *   alm_grad  device complex128, alm layout (overwritten).
 * The scatter accumulates with floating-point atomics, so the last bits vary
 * between runs.  Uses (and overwrites) the plan's transform buffers; the maps
 * made by sc_set_sky_beam are kept.  The adjoint recursion sums over rings in
 * workgroups of at most 2048 rings; longer columns (lmax >= 2048) are split
 * into ring slabs whose partial gradients are added in a fixed order, so the
 * gradient workspace grows by the slab count (ceil(rings / 2048)).
 */
int sc_convolve_adjoint(sc_plan *plan, const double *blm, const double *ptg, const void *tod_grad, int64_t n,
                        double *alm_grad);

/*
 * Adjoint with respect to the beam coefficients: for a TOD gradient y it returns
 * h_lk = dL/dRe(b_lk) + i dL/dIm(b_lk) of L = sum_t y_t c_t (h_l0 real), i.e.
 * <y, c> = Re sum_{l, k >= 0} conj(h_lk) b_lk with Im b_l0 ignored.  The TOD is
 * bilinear in (a, b): the scatter and the adjoint transforms are those of
 * sc_convolve_adjoint, and the adjoint ring sums contract with the sky instead
 * of the beam (summing over m instead of k).
 *   alm       device complex128, the sky in the plan's sky layout (SC_PARAM_SKY_LMAX).
 *   ptg       device float64 [n][3].
 *   tod_grad  device float64 [n] (SC_FP64) or float32 [n].
 *   blm_grad  device complex128, blm layout of (lmax, kmax) (overwritten).
 * Allocates (lmax+1) n_blm complex128 of plan workspace on first use.  Same
 * stream, rounding and buffer behaviour as sc_convolve_adjoint.
 */
int sc_convolve_adjoint_beam(sc_plan *plan, const double *alm, const double *ptg, const void *tod_grad, int64_t n,
                             double *blm_grad);

/*
 * Orbital dipole and quadrupole through the full beam (Galloway et al. 2022,
 * Sec. 3.3, Eqs. 14-19): for the kinematic sky D(n) = T0 [beta.n + q (beta.n)^2]
 * the convolution at pointing (theta, phi, psi) is T0 [u.S + q u^T S2 u] with
 * u = R^T beta, R = R_z(phi) R_y(theta) R_z(psi), and S, S2 the beam's first
 * and second moments in the beam frame (formed on the device from its l <= 2
 * coefficients).  No plan is needed.
 *   blm                 device complex128, layout of (lmax, kmax) as for the plans.
 *   ptg, n              device float64 [n][3] (theta, phi, psi).
 *   beta                device float64 [ceil(n / samples_per_period)][3]: v / c in the
 *                       sky frame, one entry per pointing period; sample s uses
 *                       entry s / samples_per_period.
 *   T0, q               CMB temperature and the frequency-dependent quadrupole factor.
 *   out                 device float64 [n].
 * Asynchronous on `stream`; SC_EINVAL for host or misaligned pointers or bad sizes.
 */
int sc_dipole_response(const double *blm, int lmax, int kmax, const double *ptg, int64_t n, const double *beta,
                       int64_t samples_per_period, double T0, double q, double *out, void *stream);

/*
 * Device-side numerical details for tests: copies internal stage buffers to
 * the caller's device memory.  which = 0: ring sums F (complex128
 * [kmax+1][2 lmax+1][n_rings], F_k(theta_j, m) = sum_l a_lm conj(b_lk) d^l_mk(theta_j),
 * theta_j = (j + 1/2) pi / n_rings); which = 1: the component maps in (row,
 * column, component) order (map_rows x map_cols x n_comp_padded, FP64 or FP32 by
 * precision; the maps are stored column-tiled and reordered by the copy, which is
 * enqueued on the plan's stream);
 * which = 2: the sample order of the most recent binning pass (int32, one entry
 * per sample of that pass: the index, within the pass, of the sample at each
 * position when the samples are grouped by interpolation anchor; SC_ESTATE if
 * no binned interpolation has run).
 * Returns the number of bytes copied, or a negative code.
 */
int64_t sc_debug_copy_stage(sc_plan *plan, int which, void *dst, int64_t capacity_bytes);

/*
 * Per-kernel timing.  With timing enabled the plan records a pair of HIP events
 * on its stream around every kernel launch.  sc_plan_stage_times waits for
 * the recorded events, adds each launch's duration to its stage total, writes
 * ms[s] (total milliseconds) and launches[s] for the first nstage stages, and
 * clears the records.  Stages: 0 ring sums (recursion + contraction),
 * 1 theta upsampling, 2 phi synthesis, 3 interpolation + k-sum, 4 pointing
 * binning (anchor keys, scan, scatter, work items), 5 adjoint scatter,
 * 6 adjoint transforms, 7 adjoint ring sums.
 * Returns the number of stages (8).
 */
int sc_plan_enable_timing(sc_plan *plan, int enable);
int sc_plan_stage_times(sc_plan *plan, double *ms, int64_t *launches, int nstage);

/*
 * Tunable parameters of a plan (chosen by the autotuner in the Python
 * package; defaults work everywhere).
 *   SC_PARAM_BIN_CHUNK          samples per gather/scatter work item, 16 .. 2^20 (default 256)
 *   SC_PARAM_GATHER_WGS_PER_CU  persistent gather/scatter workgroups per CU, 0 = as many as fit
 *   SC_PARAM_RING_RPT           northern rings per lane and recursion of the ring-sum kernel, 1..4
 *   SC_PARAM_SKY_LMAX           band limit of the layout of the alm array given to
 *                               sc_set_sky_beam (>= lmax; a shared sky may have a larger one)
 *   SC_PARAM_GATHER_WAVES       waves per workgroup of the SC_MMA_FP32 gather, 4 or 8 (default 4);
 *                               the same 128-sample chunk split over more waves (the split
 *                               form always runs 4)
 *   SC_PARAM_GATHER_MMA         product form of the FP32 matrix-core gather and adjoint
 *                               scatter (sc_gather_mma): SC_MMA_SPLIT16 (default) or SC_MMA_FP32
 *   SC_PARAM_VALIDATE           0 (default) or 1.  With 1, sc_set_sky_beam, sc_interpolate,
 *                               sc_interpolate_psi, sc_plan_convolve and the adjoints first count
 *                               the NaN and infinite values of their floating-point inputs on the
 *                               plan's stream and wait for the count (a host synchronisation);
 *                               any such value returns SC_EINVAL naming the input, before
 *                               anything is launched.  With 0 nothing is inspected: theta is
 *                               clamped to [0, pi], phi and psi are reduced modulo 2 pi, and a
 *                               NaN angle is read as 0.  sc_interpolate_noalloc does not
 *                               validate (the check needs a device counter).
 *   SC_PARAM_DETERMINISTIC      0 (default) or 1 (FP32-map plans with W = 8 only; SC_EINVAL
 *                               otherwise).  With 1 the adjoints' scatter uses no atomics: each
 *                               work item writes its 8 x 8 patch gradient to plan workspace
 *                               (64 x 16 ceil(ncomp/16) floats per item, allocated on first
 *                               use and kept), and every map pixel sums the patches that
 *                               cover it in a fixed order, so the gradients are bit-identical
 *                               from run to run.  It reads back the work-item count of each
 *                               binning pass (a host synchronisation).  With 0 the patches are
 *                               added with FP32 atomics (run-to-run differences at the FP32
 *                               rounding level).
 */
enum sc_param {
    SC_PARAM_BIN_CHUNK = 1,
    SC_PARAM_GATHER_WGS_PER_CU = 2,
    SC_PARAM_RING_RPT = 3,
    SC_PARAM_SKY_LMAX = 4,
    SC_PARAM_GATHER_WAVES = 5,
    SC_PARAM_GATHER_MMA = 6,
    SC_PARAM_VALIDATE = 7,
    SC_PARAM_DETERMINISTIC = 8,
    SC_PARAM_BATCH_CHAINS = 9
};

/*
 * Product forms of the interpolation contraction (FP32 maps, W = 8), both with
 * FP32 accumulation:
 *   SC_MMA_FP32     FP32 x FP32 matrix products.
 *   SC_MMA_SPLIT16  every FP32 operand split into two FP16 parts (x ~ x_hi + x_lo,
 *                   about 2^-24 relative) and each product taken as
 *                   a_hi b_hi + a_hi b_lo + a_lo b_hi on the FP16 matrix cores,
 *                   with exact power-of-two range scalings; about 3/16 of the
 *                   matrix time of SC_MMA_FP32 at a similar rounding level.
 */
enum sc_gather_mma { SC_MMA_FP32 = 0, SC_MMA_SPLIT16 = 1 };
int sc_plan_set_param(sc_plan *plan, int param, int64_t value);
int sc_plan_get_param(const sc_plan *plan, int param, int64_t *value);

/*
 * Batches: several detectors convolved with one sky (the per-detector use of
 * the method; each detector has its own beam, band limit, truncation and
 * pointing).  Each detector gets its own maps; the interpolation of all
 * detectors runs as ONE persistent launch that takes work items (samples of one
 * stencil anchor of one detector) from a shared queue.
 *
 *   lmax, kmax  the detector's beam band limit and truncation (lmax <= lmax_sky)
 *   blm         device complex128, layout of (lmax, kmax)
 *   ptg, n      device float64 [n][3], 0 <= n <= 2^27
 *   tod         device float32 [n] output
 */
typedef struct sc_det_desc {
    int lmax;
    int kmax;
    const double *blm;
    const double *ptg;
    int64_t n;
    float *tod;
} sc_det_desc;

typedef struct sc_batch sc_batch;

/* Create a batch (precision SC_F64MAPS_F32GATHER or SC_MIXED).  The descriptors
   are copied; their buffers must stay valid (contents may change) for the
   batch's lifetime. */
int sc_batch_create(sc_batch **batch, const sc_det_desc *dets, int ndet, int lmax_sky, int precision,
                    void *stream);

/* Synthesise every detector's maps from alm_sky (complex128, layout lmax_sky)
   and write every tod.  use_graph = 0: plain launches.  use_graph = 1: the first
   call runs eagerly once, then captures the whole sequence in a hipGraph and
   launches it; later calls with the same alm_sky pointer replay the graph (a
   different pointer or a parameter change re-captures). */
int sc_batch_run(sc_batch *batch, const double *alm_sky, int use_graph);

/* Tunables: det = -1 applies to every detector.  SC_PARAM_GATHER_WGS_PER_CU is
   batch-wide (the single gather launch), and so is SC_PARAM_BATCH_CHAINS: the
   detectors' map synthesis and binning run as that many independent chains (1 .. 4,
   default 4; chain 0 on the batch's stream, the others on side streams at default
   priority forked from it and joined before the gather, also inside the captured
   graph), detectors assigned by estimated work.  The outputs do not depend on it. */
int sc_batch_set_param(sc_batch *batch, int det, int param, int64_t value);
int sc_batch_get_param(const sc_batch *batch, int det, int param, int64_t *value);

/* Change the stream a batch enqueues and replays on; the new stream first waits
   for all work queued on the old one. */
int sc_batch_set_stream(sc_batch *batch, void *stream);

/* The plan of detector det (owned by the batch; for inspection and timing). */
int sc_batch_plan(sc_batch *batch, int det, sc_plan **plan);

/* Release a batch (synchronises its stream). */
int sc_batch_destroy(sc_batch *batch);

/* Human-readable text for a status code. */
const char *sc_strerror(int code);

/* Message describing the calling thread's last error (empty if none). */
const char *sc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIDELOBE_H */
