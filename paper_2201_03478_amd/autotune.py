"""Autotuner for the tunable launch parameters of a plan or a batch.

For one (lmax, kmax, precision) it times, with HIP events on the current
stream, the candidates of
  * ring_rpt           rings per lane of the ring-sum kernel (ring-sum stage time),
  * bin_chunk          samples per gather work item, and
  * gather_wgs_per_cu  persistent gather workgroups per CU and
  * gather_waves       waves per workgroup of the FP32-product gather (binning + gather time),
keeps the fastest, and caches the choice in a JSON file keyed by
"arch|L<lmax>|K<kmax>|P<precision>" ($SC_AUTOTUNE_CACHE, default
~/.cache/paper_2201_03478_amd/autotune.json).  Only launch shapes change: every
candidate computes the same result.
"""
from __future__ import annotations

import json
import os

import torch

from . import _native as N

RING_RPT = {N.SC_FP64: (1, 2, 3, 4), N.SC_F64MAPS_F32GATHER: (1, 2, 3, 4), N.SC_MIXED: (1, 2, 3, 4)}
BIN_CHUNK = (128, 256, 512, 1024)
WGS_PER_CU = (0, 1)
GATHER_WAVES = (4, 8)


def cache_path() -> str:
    return os.environ.get("SC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2201_03478_amd", "autotune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(lmax: int, kmax: int, precision: int) -> str:
    return "%s|L%d|K%d|P%d" % (_arch(), lmax, kmax, precision)


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def save_cache(c: dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_plan(plan, alm, blm, ptg, reps: int = 3, use_cache: bool = True) -> dict:
    """Choose ring_rpt, bin_chunk and gather_wgs_per_cu for plan on these inputs; apply and cache."""
    key = cache_key(plan.lmax, plan.kmax, plan.precision)
    cache = load_cache() if use_cache else {}
    if key in cache:
        best = cache[key]
    else:
        best = {}
        times = {}
        for r in RING_RPT[plan.precision]:
            try:
                plan.set_param("ring_rpt", r)
            except N.ScError:
                continue  # layout not available for this ring count
            times[r] = _time(lambda: plan.set_sky_beam(alm, blm), reps)
        best["ring_rpt"] = min(times, key=times.get)
        plan.set_param("ring_rpt", best["ring_rpt"])
        plan.set_sky_beam(alm, blm)
        out = torch.empty(ptg.shape[0], dtype=plan.tod_dtype, device=ptg.device)
        times = {}
        # the workgroup shape is a choice of the FP32 product form only
        shapes = GATHER_WAVES if plan.get_param("gather_mma") == N.SC_MMA_FP32 else (4,)
        for c in BIN_CHUNK:
            for w in WGS_PER_CU:
                for nw in shapes:
                    plan.set_param("bin_chunk", c)
                    plan.set_param("gather_wgs_per_cu", w)
                    plan.set_param("gather_waves", nw)
                    times[(c, w, nw)] = _time(lambda: plan.interpolate(ptg, out=out), reps)
        best["bin_chunk"], best["gather_wgs_per_cu"], best["gather_waves"] = min(times, key=times.get)
        if use_cache:
            cache = load_cache()
            cache[key] = best
            save_cache(cache)
    for k, v in best.items():
        plan.set_param(k, v)
    return dict(best)


def tune_batch(batch, alm_sky, reps: int = 2, use_cache: bool = True) -> list:
    """Tune each distinct (lmax, kmax) of a batch on its first detector's data; apply to all."""
    chosen = {}
    for i, d in enumerate(batch.dets):
        key = (d["lmax"], d["kmax"])
        if key not in chosen:
            p = batch.plan(i)
            chosen[key] = tune_plan(p, alm_sky, d["blm"], d["ptg"], reps=reps, use_cache=use_cache)
    wgs, waves = {}, {}
    for i, d in enumerate(batch.dets):
        best = chosen[(d["lmax"], d["kmax"])]
        batch.set_param("ring_rpt", best["ring_rpt"], det=i)
        batch.set_param("bin_chunk", best["bin_chunk"], det=i)
        n = d["ptg"].shape[0]
        wgs[best["gather_wgs_per_cu"]] = wgs.get(best["gather_wgs_per_cu"], 0) + n
        waves[best["gather_waves"]] = waves.get(best["gather_waves"], 0) + n
    # one gather launch serves all detectors: the choices covering most samples
    batch.set_param("gather_wgs_per_cu", max(wgs, key=wgs.get))
    batch.set_param("gather_waves", max(waves, key=waves.get))
    return [chosen[(d["lmax"], d["kmax"])] for d in batch.dets]
