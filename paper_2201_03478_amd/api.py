"""Python API over the C ABI: same names as the C entry points.

Tensors are torch tensors on the GPU (torch provides device memory and the
stream); the library does all of the arithmetic.  Layouts are those of
include/sidelobe.h: alm/blm complex128 m-major triangular, ptg float64 [n, 3]
(theta, phi, psi), tod float64 (SC_FP64) or float32.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N

PRECISIONS = {"fp64": N.SC_FP64, "f64maps_f32gather": N.SC_F64MAPS_F32GATHER, "mixed": N.SC_MIXED}
INFO_KEYS = ("lmax", "kmax", "precision", "W", "n_rings", "n_fft_theta", "n_theta_fine", "n_phi",
             "map_rows", "map_cols", "n_comp", "n_comp_padded", "workspace_bytes", "mid_bytes")


def n_alm(lmax: int, mmax: int | None = None) -> int:
    mmax = lmax if mmax is None else mmax
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def _prec(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptg_rows(ptg) -> int:
    """Number of pointings of a [n, 3] tensor (ValueError for any other shape)."""
    if not isinstance(ptg, torch.Tensor):
        raise TypeError("ptg must be a tensor")
    if ptg.dim() != 2 or ptg.shape[1] != 3:
        raise ValueError("ptg must be [n, 3], got %s" % (tuple(ptg.shape),))
    return ptg.shape[0]


def _numel(t, name: str, want: int):
    """Size check before any device access: the C side cannot see tensor sizes."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if t.numel() != want:
        raise ValueError("%s has %d entries, need %d" % (name, t.numel(), want))


def _dev(t: torch.Tensor, name: str, dtype) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


PARAMS = {"bin_chunk": N.SC_PARAM_BIN_CHUNK, "gather_wgs_per_cu": N.SC_PARAM_GATHER_WGS_PER_CU,
          "ring_rpt": N.SC_PARAM_RING_RPT, "sky_lmax": N.SC_PARAM_SKY_LMAX, "gather_waves": N.SC_PARAM_GATHER_WAVES,
          "gather_mma": N.SC_PARAM_GATHER_MMA, "validate": N.SC_PARAM_VALIDATE,
          "deterministic": N.SC_PARAM_DETERMINISTIC, "batch_chains": N.SC_PARAM_BATCH_CHAINS}


class Plan:
    """sc_plan: geometry, workspace and resident maps for one (lmax, kmax, precision)."""

    def __init__(self, lmax: int, kmax: int, precision="f64maps_f32gather", kernel_width: int = 0,
                 stream=None, _handle=None):
        lib = N.load()
        self._lib = lib
        self._owned = _handle is None
        if _handle is None:
            self._p = ctypes.c_void_p()
            N.check(lib.sc_plan_create(ctypes.byref(self._p), int(lmax), int(kmax), _prec(precision),
                                       int(kernel_width), ctypes.c_void_p(_stream_handle(stream))),
                    "sc_plan_create")
        else:
            self._p = _handle
        self.lmax, self.kmax = int(lmax), int(kmax)
        self.precision = _prec(precision)
        self.tod_dtype = torch.float64 if self.precision == N.SC_FP64 else torch.float32

    def close(self):
        if self._owned and getattr(self, "_p", None) and self._p.value:
            N.check(self._lib.sc_plan_destroy(self._p), "sc_plan_destroy")
            self._p = ctypes.c_void_p()

    def set_param(self, name: str, value: int):
        N.check(self._lib.sc_plan_set_param(self._p, PARAMS[name], int(value)), "sc_plan_set_param")

    def get_param(self, name: str) -> int:
        v = ctypes.c_int64()
        N.check(self._lib.sc_plan_get_param(self._p, PARAMS[name], ctypes.byref(v)), "sc_plan_get_param")
        return v.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        N.check(self._lib.sc_plan_set_stream(self._p, ctypes.c_void_p(_stream_handle(stream))),
                "sc_plan_set_stream")

    def info(self) -> dict:
        out = (ctypes.c_int64 * len(INFO_KEYS))()
        N.check(self._lib.sc_plan_info(self._p, out, len(INFO_KEYS)), "sc_plan_info")
        return dict(zip(INFO_KEYS, list(out)))

    def set_sky_beam(self, alm: torch.Tensor, blm: torch.Tensor):
        _numel(alm, "alm", n_alm(self.get_param("sky_lmax")))
        _numel(blm, "blm", n_alm(self.lmax, self.kmax))
        _dev(alm, "alm", torch.complex128)
        _dev(blm, "blm", torch.complex128)
        self.set_stream()
        N.check(self._lib.sc_set_sky_beam(self._p, alm.data_ptr(), blm.data_ptr()), "sc_set_sky_beam")
        self._keep = (alm, blm)

    def interpolate(self, ptg: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = _ptg_rows(ptg)
        if out is not None:
            _numel(out, "tod", n)
        _dev(ptg, "ptg", torch.float64)
        if out is None:
            out = torch.empty(n, dtype=self.tod_dtype, device=ptg.device)
        _dev(out, "tod", self.tod_dtype)
        self.set_stream()
        if n:
            N.check(self._lib.sc_interpolate(self._p, ptg.data_ptr(), n, out.data_ptr()), "sc_interpolate")
        return out

    def build_psi_cube(self, npsi: int = 0):
        """The paper's second step: the cube c(theta, phi, psi) from the current maps
        (npsi = 0: the smallest 2,3,5-smooth size >= 2 (2 kmax + 1))."""
        self.set_stream()
        N.check(self._lib.sc_plan_build_psi_cube(self._p, int(npsi)), "sc_plan_build_psi_cube")

    def interpolate_psi(self, ptg: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """The convolution at ptg by three-dimensional interpolation of the cube."""
        n = _ptg_rows(ptg)
        if out is not None:
            _numel(out, "tod", n)
        _dev(ptg, "ptg", torch.float64)
        if out is None:
            out = torch.empty(n, dtype=self.tod_dtype, device=ptg.device)
        _dev(out, "tod", self.tod_dtype)
        self.set_stream()
        if n:
            N.check(self._lib.sc_interpolate_psi(self._p, ptg.data_ptr(), n, out.data_ptr()), "sc_interpolate_psi")
        return out

    def convolve(self, alm: torch.Tensor, blm: torch.Tensor, ptg: torch.Tensor,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        """set_sky_beam + interpolate in one call (sc_plan_convolve: the pointing
        binning overlaps the map synthesis on a side stream)."""
        _numel(alm, "alm", n_alm(self.get_param("sky_lmax")))
        _numel(blm, "blm", n_alm(self.lmax, self.kmax))
        n = _ptg_rows(ptg)
        if out is not None:
            _numel(out, "tod", n)
        _dev(alm, "alm", torch.complex128)
        _dev(blm, "blm", torch.complex128)
        _dev(ptg, "ptg", torch.float64)
        if out is None:
            out = torch.empty(n, dtype=self.tod_dtype, device=ptg.device)
        _dev(out, "tod", self.tod_dtype)
        self.set_stream()
        N.check(self._lib.sc_plan_convolve(self._p, alm.data_ptr(), blm.data_ptr(), ptg.data_ptr(), n,
                                           out.data_ptr()), "sc_plan_convolve")
        self._keep = (alm, blm)
        return out

    def adjoint(self, blm: torch.Tensor, ptg: torch.Tensor, tod_grad: torch.Tensor,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """sc_convolve_adjoint: g_lm = dL/dRe a_lm + i dL/dIm a_lm of L = sum_t y_t c_t (complex128,
        the lmax layout of the plan, not the sky layout of a larger shared sky)."""
        _numel(blm, "blm", n_alm(self.lmax, self.kmax))
        n = _ptg_rows(ptg)
        _numel(tod_grad, "tod_grad", n)
        if out is not None:
            _numel(out, "alm_grad", n_alm(self.lmax))
        _dev(blm, "blm", torch.complex128)
        _dev(ptg, "ptg", torch.float64)
        _dev(tod_grad, "tod_grad", self.tod_dtype)
        if out is None:
            out = torch.empty(n_alm(self.lmax), dtype=torch.complex128, device=ptg.device)
        _dev(out, "alm_grad", torch.complex128)
        self.set_stream()
        N.check(self._lib.sc_convolve_adjoint(self._p, blm.data_ptr(), ptg.data_ptr(), tod_grad.data_ptr(), n,
                                              out.data_ptr()), "sc_convolve_adjoint")
        return out

    def adjoint_beam(self, alm: torch.Tensor, ptg: torch.Tensor, tod_grad: torch.Tensor,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """sc_convolve_adjoint_beam: h_lk = dL/dRe b_lk + i dL/dIm b_lk of L = sum_t y_t c_t (complex128)."""
        _numel(alm, "alm", n_alm(self.get_param("sky_lmax")))
        n = _ptg_rows(ptg)
        _numel(tod_grad, "tod_grad", n)
        if out is not None:
            _numel(out, "blm_grad", n_alm(self.lmax, self.kmax))
        _dev(alm, "alm", torch.complex128)
        _dev(ptg, "ptg", torch.float64)
        _dev(tod_grad, "tod_grad", self.tod_dtype)
        if out is None:
            out = torch.empty(n_alm(self.lmax, self.kmax), dtype=torch.complex128, device=ptg.device)
        _dev(out, "blm_grad", torch.complex128)
        self.set_stream()
        N.check(self._lib.sc_convolve_adjoint_beam(self._p, alm.data_ptr(), ptg.data_ptr(), tod_grad.data_ptr(), n,
                                                   out.data_ptr()), "sc_convolve_adjoint_beam")
        return out

    STAGES = ("ring_sums", "theta_upsample", "phi_synthesis", "gather", "binning", "scatter",
              "adjoint_transforms", "adjoint_ring_sums")

    def enable_timing(self, enable: bool = True):
        N.check(self._lib.sc_plan_enable_timing(self._p, 1 if enable else 0), "sc_plan_enable_timing")

    def stage_times(self) -> dict:
        """{stage: (total ms, launches)} from the HIP events recorded since the last call."""
        ns = len(self.STAGES)
        ms = (ctypes.c_double * ns)()
        cnt = (ctypes.c_int64 * ns)()
        N.check(self._lib.sc_plan_stage_times(self._p, ms, cnt, ns), "sc_plan_stage_times")
        return {s: (ms[i], cnt[i]) for i, s in enumerate(self.STAGES)}

    def debug_stage(self, which: int, n: int = 0) -> torch.Tensor:
        """Copy of an internal stage: 0 = ring sums F (complex128 [kmax+1, 2 lmax+1, n_rings]),
        1 = the component maps in (row, column, component) order ([map_rows, map_cols, n_comp_padded]),
        2 = the anchor-grouped sample order of the last binning pass (int32 [n], n its samples)."""
        inf = self.info()
        dev = torch.device("cuda", torch.cuda.current_device())
        if which == 2:
            t = torch.empty(n, dtype=torch.int32, device=dev)
        elif which == 0:
            t = torch.empty((self.kmax + 1, 2 * self.lmax + 1, inf["n_rings"]), dtype=torch.complex128, device=dev)
        else:
            dt = torch.float64 if self.precision == N.SC_FP64 else torch.float32
            t = torch.empty((inf["map_rows"], inf["map_cols"], inf["n_comp_padded"]), dtype=dt, device=dev)
        self.set_stream()
        N.check(self._lib.sc_debug_copy_stage(self._p, which, t.data_ptr(), t.numel() * t.element_size()),
                "sc_debug_copy_stage")
        return t


def convolve(alm: torch.Tensor, blm: torch.Tensor, lmax: int, kmax: int, ptg: torch.Tensor,
             precision="f64maps_f32gather", out: torch.Tensor | None = None) -> torch.Tensor:
    """One-shot convolve(alm, blm, lmax, kmax, pointings) -> tod (sc_convolve).

    The library caches one plan per (lmax, kmax, precision, device); release_cache()
    frees them."""
    if not (0 <= int(kmax) <= int(lmax)):
        raise ValueError("need 0 <= kmax <= lmax, got lmax=%d kmax=%d" % (lmax, kmax))
    _numel(alm, "alm", n_alm(int(lmax)))
    _numel(blm, "blm", n_alm(int(lmax), int(kmax)))
    n = _ptg_rows(ptg)
    if out is not None:
        _numel(out, "tod", n)
    lib = N.load()
    _dev(alm, "alm", torch.complex128)
    _dev(blm, "blm", torch.complex128)
    _dev(ptg, "ptg", torch.float64)
    p = _prec(precision)
    dt = torch.float64 if p == N.SC_FP64 else torch.float32
    if out is None:
        out = torch.empty(n, dtype=dt, device=ptg.device)
    _dev(out, "tod", dt)
    N.check(lib.sc_convolve(alm.data_ptr(), blm.data_ptr(), int(lmax), int(kmax), ptg.data_ptr(), n,
                            out.data_ptr(), p, ctypes.c_void_p(_stream_handle())), "sc_convolve")
    return out


def release_cache():
    """Free the plans cached by the one-shot convolve (sc_convolve_release_cache)."""
    N.check(N.load().sc_convolve_release_cache(), "sc_convolve_release_cache")


def dipole_response(blm: torch.Tensor, lmax: int, kmax: int, ptg: torch.Tensor, beta: torch.Tensor,
                    samples_per_period: int, T0: float, q: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """Orbital dipole + quadrupole through the full beam (sc_dipole_response).

    beta: float64 [ceil(n / samples_per_period), 3], v / c per pointing period."""
    n = _ptg_rows(ptg)
    _numel(blm, "blm", n_alm(lmax, kmax))
    if samples_per_period < 1:
        raise ValueError("samples_per_period must be >= 1")
    if beta.numel() < 3 * ((n + samples_per_period - 1) // samples_per_period):
        raise ValueError("beta holds too few pointing periods")
    if out is not None:
        _numel(out, "out", n)
    lib = N.load()
    _dev(blm, "blm", torch.complex128)
    _dev(ptg, "ptg", torch.float64)
    _dev(beta, "beta", torch.float64)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=ptg.device)
    _dev(out, "out", torch.float64)
    N.check(lib.sc_dipole_response(blm.data_ptr(), int(lmax), int(kmax), ptg.data_ptr(), n, beta.data_ptr(),
                                   int(samples_per_period), float(T0), float(q), out.data_ptr(),
                                   ctypes.c_void_p(_stream_handle())), "sc_dipole_response")
    return out


class SidelobeConv(torch.autograd.Function):
    """tod = A(alm) for a fixed beam and pointing; backward is the library's adjoint.

    Gradients follow torch's complex convention dL/dRe + i dL/dIm (what
    sc_convolve_adjoint returns); beam and pointing gradients are not provided.
    """

    @staticmethod
    def forward(ctx, alm, blm, ptg, plan):
        plan.set_sky_beam(alm.detach(), blm.detach())
        tod = plan.interpolate(ptg.detach())
        ctx.plan = plan
        ctx.save_for_backward(blm, ptg)
        return tod

    @staticmethod
    def backward(ctx, g):
        blm, ptg = ctx.saved_tensors
        grad = None
        if ctx.needs_input_grad[0]:
            grad = ctx.plan.adjoint(blm.detach(), ptg.detach(), g.detach().to(ctx.plan.tod_dtype).contiguous())
        return grad, None, None, None


def sidelobe_convolve(alm: torch.Tensor, blm: torch.Tensor, ptg: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable convolution (gradient with respect to alm)."""
    return SidelobeConv.apply(alm, blm, ptg, plan)


class Batch:
    """sc_batch: detectors sharing one sky; one persistent gather launch, optional hipGraph replay.

    dets: list of dicts with lmax, kmax, blm (complex128), ptg (float64 [n, 3]) and optionally
    tod (float32 [n]); outputs are written to each det's "tod" (allocated if missing).
    """

    def __init__(self, dets, lmax_sky: int, precision="f64maps_f32gather", stream=None):
        lib = N.load()
        self._lib = lib
        self.lmax_sky = int(lmax_sky)
        self.precision = _prec(precision)
        self.dets = []
        arr = (N.DetDesc * len(dets))()
        for i, d in enumerate(dets):
            blm = _dev(d["blm"], "blm", torch.complex128)
            ptg = _dev(d["ptg"], "ptg", torch.float64)
            n = ptg.shape[0]
            tod = d.get("tod")
            if tod is None:
                tod = torch.empty(n, dtype=torch.float32, device=ptg.device)
            _dev(tod, "tod", torch.float32)
            if blm.numel() != n_alm(d["lmax"], d["kmax"]) or tod.numel() != n:
                raise ValueError("detector %d: blm/tod sizes do not match" % i)
            self.dets.append(dict(lmax=int(d["lmax"]), kmax=int(d["kmax"]), blm=blm, ptg=ptg, tod=tod))
            arr[i] = N.DetDesc(int(d["lmax"]), int(d["kmax"]), blm.data_ptr(), ptg.data_ptr(), n, tod.data_ptr())
        self._b = ctypes.c_void_p()
        N.check(lib.sc_batch_create(ctypes.byref(self._b), arr, len(dets), self.lmax_sky, self.precision,
                                    ctypes.c_void_p(_stream_handle(stream))), "sc_batch_create")

    def run(self, alm_sky: torch.Tensor, use_graph: bool = True, stream=None):
        """Enqueue the batch (or replay its graph) on `stream` (default: torch's current
        stream), ordered after the batch's earlier work."""
        _numel(alm_sky, "alm_sky", n_alm(self.lmax_sky))
        _dev(alm_sky, "alm_sky", torch.complex128)
        N.check(self._lib.sc_batch_set_stream(self._b, ctypes.c_void_p(_stream_handle(stream))),
                "sc_batch_set_stream")
        self._sky = alm_sky
        N.check(self._lib.sc_batch_run(self._b, alm_sky.data_ptr(), 1 if use_graph else 0), "sc_batch_run")
        return [d["tod"] for d in self.dets]

    def set_param(self, name: str, value: int, det: int = -1):
        N.check(self._lib.sc_batch_set_param(self._b, int(det), PARAMS[name], int(value)), "sc_batch_set_param")

    def get_param(self, name: str, det: int = 0) -> int:
        v = ctypes.c_int64()
        N.check(self._lib.sc_batch_get_param(self._b, int(det), PARAMS[name], ctypes.byref(v)),
                "sc_batch_get_param")
        return v.value

    def plan(self, det: int) -> Plan:
        """Non-owning view of detector det's plan (its sky layout is lmax_sky)."""
        h = ctypes.c_void_p()
        N.check(self._lib.sc_batch_plan(self._b, int(det), ctypes.byref(h)), "sc_batch_plan")
        d = self.dets[det]
        return Plan(d["lmax"], d["kmax"], self.precision, _handle=h)

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            N.check(self._lib.sc_batch_destroy(self._b), "sc_batch_destroy")
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
