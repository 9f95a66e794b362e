#!/usr/bin/env python3
"""Benchmark: convolved TOD samples/s at lmax 512, kmax 100 on one MI355X.

One step is the whole hot path on one batch of synthetic input already
resident in HBM: map synthesis from (a_lm, b_lk) (ring sums by Wigner-d
recursion, theta upsampling, phi synthesis) and the interpolation + k-sum at
every pointing of a 1e7-sample synthetic scan.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--precision f64maps_f32gather|fp64]

Per-kernel durations come from HIP events the library records on its streams
around each launch, in a second pass of the same steps after the timed ones
(the timed steps run without those events); the roofline object uses the
dominant kernel of the plan's own stream (the pointing binning runs beside the
map synthesis on a side stream).  The CPU baseline is the oracle (direct sum of Eq. 2) timed on
a bounded random sample of the same pointings; its outputs also give the GPU
result's error.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "conv TOD samples/s, lmax512 kmax100, mixed vs FP64 at 1e-6 rel err"
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "fp16": 2.5e15, "hbm": 8.0e12}  # MI355X published (dense) peaks
# The split gather forms one FP32-accurate product block from four FP16 matrix
# products and one FP8 product (half the FP16 time): 4.5 FP16 blocks.
PEAK["split"] = PEAK["fp16"] / 4.5

# Sources each stage's kernels are built from (their traffic records are tied to these).
STAGE_SOURCES = {
    "ring_sums": ["k_synth.hip", "wigner_rec.h"],
    "theta_upsample": ["k_fft.hip", "fft_lds.h"],
    "phi_synthesis": ["k_fft.hip", "fft_lds.h"],
    "gather": ["k_gather.hip"],
    "binning": ["k_bin.hip"],
}


def ring_dvalues(L: int, K: int, nring: int) -> int:
    """Number of Wigner-d values the ring-sum kernel evaluates (l >= max(m, k), m, k >= 0)."""
    tot = 0
    for k in range(K + 1):
        for m in range(L + 1):
            tot += max(0, L - max(m, k) + 1)
    return tot * nring


def stage_model(info: dict, n: int, prec: int, mma: int = 1):
    """Algorithmic work per launch of each kernel: (bound, units, unit_name, peak).

    mma is the gather's product form (0: FP32 matrix products, 1: split FP16/FP8)."""
    L, K = info["lmax"], info["kmax"]
    nm = 2 * L + 1
    nr, rows, cols, Wd = info["n_rings"], info["map_rows"], info["map_cols"], info["W"]
    nc = 2 * K + 1  # algorithmic component count (the stored zero sin 0 psi map is not counted)
    esz = 8 if prec == 0 else 4
    csz = info["mid_bytes"]  # bytes per complex value of F and G (complex128 or complex64)
    dv = ring_dvalues(L, K, nr)
    return {
        # 2 FMA recursion (normalised three-term form) + 4 FMA contraction (both signs of m) per d value
        "ring_sums": ("alu", 12.0 * dv, "TFLOP/s", PEAK["fp64"]),
        # read F, write the upsampled spectra
        "theta_upsample": ("hbm", csz * (K + 1) * nm * (nr + rows), "GB/s", PEAK["hbm"]),
        # read the spectra, write the real components of the maps
        "phi_synthesis": ("hbm", csz * (K + 1) * rows * nm + esz * rows * cols * nc, "GB/s", PEAK["hbm"]),
        # one FMA per (tap, component) per sample: FP64, FP32 or split matrix products
        "gather": (("mfma", 2.0 * nc * Wd * Wd * n, "TFLOP/s", PEAK["fp64"]) if prec == 0 else
                   ("mfma", 2.0 * nc * Wd * Wd * n, "TFLOP/s", PEAK["split"] if mma == 1 else PEAK["fp32"])),
        # pointings read twice (keys, scatter), key + rank written and read, sorted record written
        "binning": ("hbm", n * (2 * 24.0 + 2 * 8.0 + 28.0), "GB/s", PEAK["hbm"]),
        # adjoint: the transpose of the gather (same products), of the transforms (map
        # gradients read, complex128 G written and read, F written) and of the ring sums
        "scatter": (("alu", 2.0 * nc * Wd * Wd * n, "TFLOP/s", PEAK["fp64"]) if prec == 0 else
                    ("mfma", 2.0 * nc * Wd * Wd * n, "TFLOP/s", PEAK["split"] if mma == 1 else PEAK["fp32"])),
        "adjoint_transforms": ("hbm", esz * rows * cols * nc + 16.0 * (K + 1) * nm * (2 * rows + nr), "GB/s",
                               PEAK["hbm"]),
        "adjoint_ring_sums": ("alu", 12.0 * dv, "TFLOP/s", PEAK["fp64"]),
    }


def rooflines(model: dict, per_launch: dict, overlapped=()) -> dict:
    """Achieved vs peak per stage from its algorithmic work per launch and launch time (ms)."""
    out = {}
    for s_, t_ in per_launch.items():
        if not t_ or s_ not in model:
            continue
        b_, u_, un_, pk_ = model[s_]
        a_ = u_ / (t_ * 1e-3)
        sc_ = 1e12 if un_ == "TFLOP/s" else 1e9
        out[s_] = {"bound": b_, "achieved": a_ / sc_, "peak": pk_ / sc_, "unit": un_, "frac": a_ / pk_,
                   "avg_launch_ms": t_}
        if s_ in overlapped:
            out[s_]["overlapped"] = "side stream, concurrent with the map synthesis (span includes waits)"
    return out


def kernel_source_hash(stage: str) -> str:
    """Hash of the sources a stage's kernels are compiled from (with the shared headers)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2201_03478_amd", "csrc")
    for f in STAGE_SOURCES[stage] + ["sc_common.h"]:
        h.update(open(os.path.join(d, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "sidelobe.h"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(stage: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they match this source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        ent = rec.get(workload, {}).get(stage)
        if ent and ent.get("source_hash") == kernel_source_hash(stage):
            return ent["bytes_per_launch"]
    except Exception:
        return None
    return None


def run_form(torch, api, dev, a, b, ptg, L, K, precision, width, steps, warmup):
    plan = api.Plan(L, K, precision, kernel_width=width)
    n = ptg.shape[0]
    tod = torch.empty(n, dtype=plan.tod_dtype, device=dev)

    def step():
        # maps from (a, b), then the TOD at ptg; the pointing binning overlaps the maps
        plan.convolve(a, b, ptg, out=tod)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # Per-stage launch times from a second pass of the same steps with the library's
    # stage events on (the events sit between the launches, so the timed steps above
    # run without them).
    plan.enable_timing(True)
    plan.stage_times()  # clear
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.enable_timing(False)
    return plan, tod, ms, stages


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f64maps_f32gather", choices=["f64maps_f32gather", "fp64"])
    ap.add_argument("--width", type=int, default=8, help="interpolation kernel width W (8 meets 1e-6)")
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: 200 samples, about 20 s)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--extras", default="", metavar="NAMES",
                    help="comma-separated subset of the other workloads to run (default: all)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, adjoint and batched workloads (extra objects in the JSON line)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n}))
        return

    import workloads as W
    from paper_2201_03478_amd import api
    from paper_2201_03478_amd import _native as N

    dev = torch.device("cuda", 0)
    cfg = W.CONFIGS["sidelobe-lmax512-kmax100"]
    L, K, n = cfg["lmax"], cfg["kmax"], args.samples
    a_np = W.sky_alm(L, W.config_seed(2, 1))
    b_np = W.beam_alm(L, K, W.config_seed(2, 2), kind="sidelobe")
    a = torch.from_numpy(a_np).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    ptg = W.scan_pointings(n, device=dev)
    torch.cuda.synchronize()
    print("bench: inputs ready (lmax %d kmax %d n %d)" % (L, K, n), file=sys.stderr, flush=True)

    plan, tod, ms, stages = run_form(torch, api, dev, a, b, ptg, L, K, args.precision, args.width,
                                     args.steps, args.warmup)
    info = plan.info()
    prec = info["precision"]
    print("bench: main form %.3f ms/step" % ms, file=sys.stderr, flush=True)

    model = stage_model(info, n, prec, plan.get_param("gather_mma"))
    per_launch = {s: (t / c if c else 0.0) for s, (t, c) in stages.items()}
    # The binning runs on the plan's side stream beside the map synthesis
    # (sc_plan_convolve): its events span the time it waits for compute units, and
    # it is off the critical path, so the dominant kernel is taken among the rest.
    OVERLAPPED = ("binning",)
    dom = max((s_ for s_ in per_launch if s_ not in OVERLAPPED), key=per_launch.get)
    bound, units, unit, peak = model[dom]
    achieved = units / (per_launch[dom] * 1e-3)
    workload_name = "sidelobe-lmax512-kmax100-scan1e7"
    traffic = measured_traffic(dom, workload_name)
    roofline = {
        "kernel": dom,
        "bound": bound,
        "achieved": achieved / 1e12 if unit == "TFLOP/s" else achieved / 1e9,
        "peak": peak / 1e12 if unit == "TFLOP/s" else peak / 1e9,
        "unit": unit,
        "frac": achieved / peak,
        "traffic": traffic,
        "avg_launch_ms": per_launch[dom],
        "algorithmic_per_launch": units,
    }

    stage_roofline = rooflines(model, per_launch, OVERLAPPED)

    result = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # FP64 synthesis; the FP32-map gather's products are split FP16/FP8 (FP32-accurate, FP32 accumulation)
        "dtype": ("f64+f16/f8split" if plan.get_param("gather_mma") == N.SC_MMA_SPLIT16 else "f64+f32")
        if prec == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": workload_name,
            "lmax": L, "kmax": K, "n_samples": n,
            "precision": args.precision, "W": info["W"],
            "grid": [info["map_rows"], info["map_cols"], info["n_comp"]],
        },
        "stages_ms_per_step": {s: t / args.steps for s, (t, c) in stages.items()},
        "roofline": roofline,
        "stage_roofline": stage_roofline,
    }

    # steady state with the maps already built (binning + gather only)
    ms_g = _event_ms(torch, lambda: plan.interpolate(ptg, out=tod), args.steps)
    result["gather_only"] = {"ms_per_step": ms_g, "value": n / (ms_g * 1e-3)}

    # oracle on a bounded random sample: CPU baseline and the error of this run
    sel = np.sort(np.random.default_rng(W.config_seed(2, 6)).choice(n, 4096, replace=False))
    if not args.no_cpu_baseline:
        import oracle
        host = host_info()
        threads = host["threads_used"]
        m = args.cpu_sample or 200
        idx = sel[:m]
        sub = ptg[torch.as_tensor(idx, device=dev)].cpu().numpy()
        got = tod[torch.as_tensor(idx, device=dev)].double().cpu().numpy()
        t0 = time.perf_counter()
        ref = oracle.convolve(a_np, b_np, L, K, sub, nthreads=threads)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": m / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded random samples of the 1e7-sample scan (%.1f s), direct sum of Eq. 2 in long "
                      "double, OpenMP over samples" % (m, dt),
            "host": host,
        }
        result["rel_err_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["max_err_vs_oracle"] = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        print("bench: oracle %d samples in %.1f s on %d threads, rel err %.2e, max %.2e"
              % (m, dt, threads, result["rel_err_vs_oracle"], result["max_err_vs_oracle"]), file=sys.stderr, flush=True)
        ref_sub, idx_sub = ref, idx
        m1 = 4
        t0 = time.perf_counter()
        oracle.convolve(a_np, b_np, L, K, sub[:m1], nthreads=1)
        result["cpu_baseline_1core"] = {"value": m1 / (time.perf_counter() - t0), "unit": "samples/s", "cores": 1,
                                        "kind": "oracle", "sample": "the first %d of the samples above" % m1}
    del plan, tod

    if not args.no_fp64_form and args.precision != "fp64":
        # the plain FP64 GPU form: at the same W = 8 (the 1e-6 target of the metric) and at its
        # own 1e-12 width (W = 14); the speed-up of the headline form is quoted against both
        fsteps = max(1, args.steps // 2)
        for key, width in (("fp64_form", args.width), ("fp64_w14_form", 14)):
            p64, tod64, ms64, st64 = run_form(torch, api, dev, a, b, ptg, L, K, "fp64", width, fsteps, 1)
            inf64 = p64.info()
            form = {"precision": "fp64", "W": inf64["W"], "ms_per_step": ms64, "value": n / (ms64 * 1e-3),
                    "stages_ms_per_step": {s: t / fsteps for s, (t, c) in st64.items() if c}}
            m64 = stage_model(inf64, n, inf64["precision"])
            g_ms = st64["gather"][0] / max(1, st64["gather"][1])
            if g_ms:
                _, u_, _, pk_ = m64["gather"]
                form["gather_roofline"] = {"bound": "mfma", "achieved": u_ / (g_ms * 1e-3) / 1e12,
                                           "peak": pk_ / 1e12, "unit": "TFLOP/s",
                                           "frac": u_ / (g_ms * 1e-3) / pk_, "avg_launch_ms": g_ms}
            if not args.no_cpu_baseline:
                got64 = tod64[torch.as_tensor(idx_sub, device=dev)].cpu().numpy()
                form["rel_err_vs_oracle"] = float(np.linalg.norm(got64 - ref_sub) / np.linalg.norm(ref_sub))
                form["max_err_vs_oracle"] = float(np.max(np.abs(got64 - ref_sub)) / np.max(np.abs(ref_sub)))
            result[key] = form
            del p64, tod64
        result["speedup_vs_fp64_form"] = result["fp64_form"]["ms_per_step"] / ms
        result["speedup_vs_fp64_w14_form"] = result["fp64_w14_form"]["ms_per_step"] / ms
        print("bench: fp64 forms done", file=sys.stderr, flush=True)

    if not args.no_extras:
        for name, fn in (("precision_variant", extra_precision), ("adjoint", extra_adjoint),
                         ("batched", extra_batched), ("dipole", extra_dipole), ("psi_cube", extra_psi_cube)):
            if args.extras and name not in args.extras.split(","):
                continue
            try:
                result[name] = fn(torch, api, W, dev, args.no_cpu_baseline)
            except Exception as exc:  # an extra must not lose the headline line
                result[name] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            torch.cuda.empty_cache()
            print("bench: %s done" % name, file=sys.stderr, flush=True)

    print(json.dumps(result), flush=True)


def host_info() -> dict:
    """The host CPU the oracle runs on: model, core counts, and the threads it is given (the
    CPU share of one GPU on the benchmark machines is 16 threads, whatever the machine has)."""
    import platform
    import subprocess
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except Exception:
        nproc = os.cpu_count() or 1
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"lscpu_model": model, "nproc": nproc, "os_cpu_count": os.cpu_count(), "affinity": aff,
            "threads_used": max(1, min(aff, nproc, 16))}


def _event_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _oracle_err(W, torch, dev, a_np, b_np, L, K, ptg, tod, m, seed):
    import oracle
    n = ptg.shape[0]
    idx = torch.as_tensor(np.sort(np.random.default_rng(seed).choice(n, m, replace=False)), device=dev)
    ref = oracle.convolve(a_np, b_np, L, K, ptg[idx].cpu().numpy(), nthreads=min(os.cpu_count() or 1, 16))
    got = tod[idx].double().cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def extra_precision(torch, api, W, dev, no_oracle):
    """lmax 1024, kmax 16, 1e8 scan samples: mixed form vs the FP64-recursion form."""
    cfg = W.CONFIGS["precision-lmax1024-kmax16"]
    L, K, n = cfg["lmax"], cfg["kmax"], cfg["n"]
    a_np, b_np = W.sky_alm(L, W.config_seed(3, 1)), W.beam_alm(L, K, W.config_seed(3, 2))
    a, b = torch.from_numpy(a_np).to(dev), torch.from_numpy(b_np).to(dev)
    ptg = W.scan_pointings(n, device=dev)
    out = {"workload": "precision-lmax1024-kmax16-scan1e8", "n_samples": n}
    for prec in ("mixed", "f64maps_f32gather"):
        plan, tod, ms, stages = run_form(torch, api, dev, a, b, ptg, L, K, prec, 8, 3, 1)
        rec = {"ms_per_step": ms, "value": n / (ms * 1e-3),
               "stages_ms_per_step": {k: t / 3 for k, (t, c) in stages.items() if c}}
        # the mixed form's ring sums are priced at the FP64 form's 12 flop per d value
        inf = plan.info()
        rec["stage_roofline"] = rooflines(stage_model(inf, n, inf["precision"], plan.get_param("gather_mma")),
                                          {k: t / c for k, (t, c) in stages.items() if c}, ("binning",))
        if not no_oracle:
            rec["rel_err_vs_oracle"] = _oracle_err(W, torch, dev, a_np, b_np, L, K, ptg, tod, 8, W.config_seed(3, 6))
        out[prec] = rec
        del plan, tod
    return out


def extra_adjoint(torch, api, W, dev, no_oracle):
    """lmax 512, kmax 32, 1e8 scan samples: forward and adjoint, with the dot-product test."""
    cfg = W.CONFIGS["adjoint-lmax512-kmax32"]
    L, K, n = cfg["lmax"], cfg["kmax"], cfg["n"]
    a_np, b_np = W.sky_alm(L, W.config_seed(5, 1)), W.beam_alm(L, K, W.config_seed(5, 2))
    a, b = torch.from_numpy(a_np).to(dev), torch.from_numpy(b_np).to(dev)
    ptg = W.scan_pointings(n, device=dev)
    y = torch.randn(n, generator=torch.Generator(device=dev).manual_seed(W.config_seed(5, 4)), device=dev)
    plan = api.Plan(L, K, "f64maps_f32gather")
    tod = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty_like(a)

    def fwd():
        plan.convolve(a, b, ptg, out=tod)

    def adj():
        plan.adjoint(b, ptg, y, out=grad)

    fms = _event_ms(torch, fwd, 3)
    ams = _event_ms(torch, adj, 3)
    plan.enable_timing(True)  # per-stage launch times from a separate pass
    plan.stage_times()
    for _ in range(3):
        adj()
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.enable_timing(False)
    fwd()
    lhs = float(torch.dot(tod.double(), y.double()))
    rhs = float(torch.sum(torch.conj(grad) * a).real)
    # gradient with respect to the beam (same scatter and transforms, contraction with the sky)
    bgrad = torch.empty_like(b)
    bms = _event_ms(torch, lambda: plan.adjoint_beam(a, ptg, y, out=bgrad), 3)
    b_real0 = b.clone()
    b_real0[:L + 1] = b_real0[:L + 1].real.to(b.dtype)
    rhs_b = float(torch.sum(torch.conj(bgrad) * b_real0).real)
    inf = plan.info()
    adj_roof = rooflines(stage_model(inf, n, inf["precision"], plan.get_param("gather_mma")),
                         {k: t / c for k, (t, c) in st.items() if c})
    return {"workload": "adjoint-lmax512-kmax32-scan1e8", "n_samples": n,
            "forward_ms": fms, "adjoint_ms": ams, "adjoint_value": n / (ams * 1e-3),
            "adjoint_stages_ms": {k: t / 4 for k, (t, c) in st.items() if c},
            "adjoint_stage_roofline": adj_roof,
            "dot_test_rel": abs(lhs - rhs) / abs(lhs),
            "beam_adjoint_ms": bms, "beam_dot_test_rel": abs(lhs - rhs_b) / abs(lhs)}


def extra_dipole(torch, api, W, dev, no_oracle):
    """Orbital dipole + quadrupole response (Sec. 3.3) on the 1e7-sample scan: one velocity per
    hour of samples; HBM-bound (24 B of pointing read and 8 B written per sample)."""
    cfg = W.CONFIGS["sidelobe-lmax512-kmax100"]
    L, K, n = cfg["lmax"], cfg["kmax"], cfg["n"]
    b = torch.from_numpy(W.beam_alm(L, K, W.config_seed(2, 2), kind="sidelobe")).to(dev)
    ptg = W.scan_pointings(n, device=dev)
    spp = 117_000  # one hour at 32.5 Hz
    nper = (n + spp - 1) // spp
    g = torch.Generator(device=dev).manual_seed(W.config_seed(2, 7))
    beta = 1e-4 * torch.randn((nper, 3), generator=g, device=dev, dtype=torch.float64)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    ms = _event_ms(torch, lambda: api.dipole_response(b, L, K, ptg, beta, spp, 2.7255, 1.25, out=out), 20)
    bytes_per = 32.0 * n
    return {"workload": "dipole-scan1e7", "n_samples": n, "ms": ms, "value": n / (ms * 1e-3),
            "unit": "samples/s", "roofline": {"bound": "hbm", "achieved": bytes_per / (ms * 1e-3) / 1e9,
                                              "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                                              "frac": bytes_per / (ms * 1e-3) / PEAK["hbm"]}}


def _next_smooth(n):
    def smooth(m):
        for q in (2, 3, 5):
            while m % q == 0:
                m //= q
        return m == 1
    while not smooth(n):
        n += 1
    return n


def extra_psi_cube(torch, api, W, dev, no_oracle):
    """The paper's second step on the lmax 512 / kmax 100 workload: the psi cube built from the
    maps (one inverse FFT over k per pixel pair), then W^3 interpolation per sample on the 1e7
    scan samples; compared with the exact cos/sin k-sum gather on the same maps."""
    cfg = W.CONFIGS["sidelobe-lmax512-kmax100"]
    L, K, n = cfg["lmax"], cfg["kmax"], cfg["n"]
    a_np = W.sky_alm(L, W.config_seed(2, 1))
    b_np = W.beam_alm(L, K, W.config_seed(2, 2), kind="sidelobe")
    plan = api.Plan(L, K, "f64maps_f32gather")
    plan.set_sky_beam(torch.from_numpy(a_np).to(dev), torch.from_numpy(b_np).to(dev))
    ptg = W.scan_pointings(n, device=dev)
    info = plan.info()
    Wk = 8
    npsi = _next_smooth(max(2 * (2 * K + 1), 2 * Wk))
    npst = (npsi + Wk - 1 + 3) // 4 * 4
    cube_ms = _event_ms(torch, lambda: plan.build_psi_cube(), 5)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    gather_ms = _event_ms(torch, lambda: plan.interpolate_psi(ptg, out=out), 5)
    exact = torch.empty(n, dtype=torch.float32, device=dev)
    ksum_ms = _event_ms(torch, lambda: plan.interpolate(ptg, out=exact), 5)
    d = float(torch.linalg.vector_norm((out - exact).double()) / torch.linalg.vector_norm(exact.double()))
    npix = info["map_rows"] * info["map_cols"]
    cube_bytes = 4.0 * npix * ((2 * K + 2) + npst)  # component maps read, cube written
    res = {"workload": "psi-cube-lmax512-kmax100-scan1e7", "n_samples": n, "npsi": npsi,
           "cube_gb": 4.0 * npix * npst / 1e9, "cube_build_ms": cube_ms, "gather_ms": gather_ms,
           "value": n / (gather_ms * 1e-3), "unit": "samples/s", "ksum_gather_ms": ksum_ms,
           "rel_l2_vs_ksum_path": d,
           "cube_roofline": {"bound": "hbm", "achieved": cube_bytes / (cube_ms * 1e-3) / 1e9,
                             "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                             "frac": cube_bytes / (cube_ms * 1e-3) / PEAK["hbm"]},
           "gather_fma_per_sample": Wk ** 3 + Wk ** 2 + Wk}
    if not no_oracle:
        res["rel_err_vs_oracle"] = _oracle_err(W, torch, dev, a_np, b_np, L, K, ptg, out, 16, W.config_seed(2, 8))
    plan.close()
    del ptg, out, exact
    torch.cuda.empty_cache()
    res["many_samples"] = _psi_many_samples(torch, api, W, dev, no_oracle)
    return res


def _psi_many_samples(torch, api, W, dev, no_oracle):
    """lmax 1024, kmax 16, 1e8 scan samples: many samples per map set and a small kmax, where the cube's
    W^3 + W^2 + W = 584 FMA per sample undercut the k-sum's (2 kmax + 1) W^2 = 2112."""
    cfg = W.CONFIGS["precision-lmax1024-kmax16"]
    L, K, n = cfg["lmax"], cfg["kmax"], cfg["n"]
    a_np, b_np = W.sky_alm(L, W.config_seed(3, 1)), W.beam_alm(L, K, W.config_seed(3, 2))
    plan = api.Plan(L, K, "f64maps_f32gather")
    plan.set_sky_beam(torch.from_numpy(a_np).to(dev), torch.from_numpy(b_np).to(dev))
    ptg = W.scan_pointings(n, device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    exact = torch.empty(n, dtype=torch.float32, device=dev)
    cube_ms = _event_ms(torch, lambda: plan.build_psi_cube(), 3)
    gather_ms = _event_ms(torch, lambda: plan.interpolate_psi(ptg, out=out), 3)
    ksum_ms = _event_ms(torch, lambda: plan.interpolate(ptg, out=exact), 3)
    d = float(torch.linalg.vector_norm((out - exact).double()) / torch.linalg.vector_norm(exact.double()))
    res = {"workload": "psi-cube-lmax1024-kmax16-scan1e8", "n_samples": n,
           "npsi": _next_smooth(max(2 * (2 * K + 1), 16)), "cube_build_ms": cube_ms, "gather_ms": gather_ms,
           "ksum_gather_ms": ksum_ms, "cube_plus_gather_ms": cube_ms + gather_ms,
           "value": n / ((cube_ms + gather_ms) * 1e-3), "unit": "samples/s", "rel_l2_vs_ksum_path": d}
    if not no_oracle:
        res["rel_err_vs_oracle"] = _oracle_err(W, torch, dev, a_np, b_np, L, K, ptg, out, 8, W.config_seed(3, 8))
    plan.close()
    return res


def extra_batched(torch, api, W, dev, no_oracle):
    """12 detectors (lmax 256/512/1024, kmax 8/32/100, 4e7 scan samples), autotuned, one gather launch."""
    from paper_2201_03478_amd import autotune
    sky = torch.from_numpy(W.sky_alm(1024, W.config_seed(4, 1))).to(dev)
    dets = []
    for i, (L, K, n) in enumerate(W.DETECTORS):
        dets.append(dict(lmax=L, kmax=K, blm=torch.from_numpy(W.beam_alm(L, K, W.config_seed(4, 10 + i))).to(dev),
                         ptg=W.scan_pointings(n, t0=1000.0 * i, psi0=i * math.pi / 12, device=dev)))
    ntot = sum(d["ptg"].shape[0] for d in dets)
    bt = api.Batch(dets, 1024)
    eager_default = _event_ms(torch, lambda: bt.run(sky, use_graph=False), 2)
    chosen = autotune.tune_batch(bt, sky, reps=2)
    eager = _event_ms(torch, lambda: bt.run(sky, use_graph=False), 3)
    graph = _event_ms(torch, lambda: bt.run(sky, use_graph=True), 3)
    # Per-stage kernel time of one eager pass with one synthesis chain (the launches run
    # one after another, so each launch's time is its own), summed over the detectors,
    # with the rooflines of those sums; and the same pass with the four chains.
    views = [bt.plan(d) for d in range(len(dets))]

    def stage_sums():
        for v in views:
            v.enable_timing(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        bt.run(sky, use_graph=False)
        t1.record()
        torch.cuda.synchronize()
        sums = {}
        for v in views:
            for name, (ms_, cnt) in v.stage_times().items():
                if cnt:
                    sums[name] = sums.get(name, 0.0) + ms_
            v.enable_timing(False)
        return sums, t0.elapsed_time(t1)

    bt.set_param("batch_chains", 1)
    serial, serial_ms = stage_sums()
    bt.set_param("batch_chains", 4)
    chained, chained_ms = stage_sums()
    units = {}
    for d, v in enumerate(views):
        inf = v.info()
        for name, (b_, u_, un_, pk_) in stage_model(inf, dets[d]["ptg"].shape[0], inf["precision"]).items():
            units[name] = (b_, units.get(name, (b_, 0.0))[1] + u_, un_, pk_)
    units["gather"] = units["gather"][:3] + (PEAK["split"],)
    batch_roof = rooflines(units, serial)
    out = {"workload": "batched-12det-scan4e7", "n_samples": ntot, "ms_per_step_graph": graph,
           "value": ntot / (graph * 1e-3), "ms_per_step_eager": eager, "ms_per_step_eager_untuned": eager_default,
           "synthesis_chains": 4, "eager_pass_ms_one_chain": serial_ms, "eager_pass_ms_four_chains": chained_ms,
           "stage_kernel_ms_one_chain": {k: round(v, 3) for k, v in serial.items()},
           "stage_kernel_ms_four_chains": {k: round(v, 3) for k, v in chained.items()},
           "stage_roofline_one_chain": batch_roof,
           "tuned": [dict(det=i, lmax=d["lmax"], kmax=d["kmax"], **c) for i, (d, c) in enumerate(zip(bt.dets, chosen))]}
    bt.close()
    return out


if __name__ == "__main__":
    main()
