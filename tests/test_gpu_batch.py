"""Batched detectors: one shared sky, per-detector beams/band limits/pointings,
one persistent gather launch, hipGraph capture and replay, the autotuner.

Each detector is the convolution of Eq. 2 (Galloway et al. 2022, Sec. 2.1) with
its own beam; the batch must give exactly what separate plans give (same
kernels and per-sample arithmetic), and match the oracle to the FP32-form bar.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_parity, coef_hash, load_golden, place_golden
from workloads.generators import truncate_alm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()
    return torch, api, torch.device("cuda", 0)


def _to(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


SMALL = [(64, 8, 3000), (40, 32, 2500), (32, 4, 1000), (80, 0, 777), (48, 20, 0)]


def _small_batch(torch, dev, lmax_sky=80):
    dets = []
    for i, (L, K, n) in enumerate(SMALL):
        p = W.uniform_pointings(n, 500 + i)
        if n:
            p[0] = [0.0, 1.0, 2.0]
        dets.append(dict(lmax=L, kmax=K, blm=_to(torch, dev, W.beam_alm(L, K, 600 + i)),
                         ptg=_to(torch, dev, p.reshape(-1, 3))))
    sky = _to(torch, dev, W.sky_alm(lmax_sky, 700))
    return dets, sky


def _single(torch, api, d, sky, lmax_sky):
    plan = api.Plan(d["lmax"], d["kmax"])
    plan.set_param("sky_lmax", lmax_sky)
    plan.set_sky_beam(sky, d["blm"])
    return plan.interpolate(d["ptg"])


def test_batch_equals_separate_plans(env):
    torch, api, dev = env
    dets, sky = _small_batch(torch, dev)
    b = api.Batch(dets, 80)
    outs = [t.clone() for t in b.run(sky, use_graph=False)]
    torch.cuda.synchronize()
    for d, o in zip(b.dets, outs):
        ref = _single(torch, api, d, sky, 80)
        torch.cuda.synchronize()
        assert torch.equal(o, ref), (d["lmax"], d["kmax"])


def test_batch_graph_replays_match_eager(env):
    """Replays interleaved with eager work; the captured graph reads the current sky contents."""
    torch, api, dev = env
    dets, sky = _small_batch(torch, dev)
    b = api.Batch(dets, 80)
    for rep in range(4):
        if rep:
            sky.mul_(1.25)  # same buffer, new contents
        graph_out = [t.clone() for t in b.run(sky, use_graph=True)]
        torch.cuda.synchronize()
        eager_out = [t.clone() for t in b.run(sky, use_graph=False)]
        torch.cuda.synchronize()
        for g, e in zip(graph_out, eager_out):
            assert torch.equal(g, e), rep


def test_batch_matches_oracle_and_autotune_keeps_results(env, oracle_lib, tmp_path):
    torch, api, dev = env
    from paper_2201_03478_amd import autotune
    dets, sky = _small_batch(torch, dev)
    b = api.Batch(dets, 80)
    before = [t.clone() for t in b.run(sky, use_graph=False)]
    torch.cuda.synchronize()
    sky_np = sky.cpu().numpy()
    for d, o in zip(b.dets, before):
        if d["ptg"].shape[0] == 0:
            continue
        ref = oracle_lib.convolve(truncate_alm(sky_np, 80, d["lmax"]), d["blm"].cpu().numpy(), d["lmax"],
                                  d["kmax"], d["ptg"].cpu().numpy())
        assert_parity(o.double().cpu().numpy(), ref, 1e-6, "small batch L=%d K=%d" % (d["lmax"], d["kmax"]))
    os.environ["SC_AUTOTUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        chosen = autotune.tune_batch(b, sky, reps=1)
    finally:
        os.environ.pop("SC_AUTOTUNE_CACHE")
    assert len(chosen) == len(SMALL)
    after = [t.clone() for t in b.run(sky, use_graph=True)]
    torch.cuda.synchronize()
    for x, y in zip(before, after):
        assert torch.equal(x, y)


def test_batched_workload_full_size(env):
    """12 detectors, lmax in {256, 512, 1024}, kmax in {8, 32, 100}, 4e7 scan samples in one
    persistent launch (hipGraph replay); 50 stored oracle samples per detector."""
    torch, api, dev = env
    golden = load_golden("batched-12det-scan4e7")
    sky_np = W.sky_alm(1024, W.config_seed(4, 1))
    sky = _to(torch, dev, sky_np)
    dets, its = [], []
    for i, (L, K, n) in enumerate(W.DETECTORS):
        g = golden[i]
        assert (g["lmax"], g["kmax"], g["n"]) == (L, K, n)
        b_np = W.beam_alm(L, K, W.config_seed(4, 10 + i))
        assert coef_hash(truncate_alm(sky_np, 1024, L), b_np) == g["coef_sha"]
        ptg = W.scan_pointings(n, t0=1000.0 * i, psi0=i * math.pi / 12, device=dev)
        its.append(place_golden(torch, ptg, g))
        dets.append(dict(lmax=L, kmax=K, blm=_to(torch, dev, b_np), ptg=ptg))
    b = api.Batch(dets, 1024)
    b.run(sky, use_graph=True)  # eager pass + capture + replay
    b.run(sky, use_graph=True)  # replay
    torch.cuda.synchronize()
    for i, d in enumerate(b.dets):
        assert_parity(d["tod"][its[i]].double().cpu().numpy(), golden[i]["c"], 1e-6,
                      "detector %d (lmax %d kmax %d n %d)" % (i, d["lmax"], d["kmax"], d["ptg"].shape[0]))


def test_batch_stage_timing_leaves_results(env):
    """Stage timing on the detectors' plans (events on each synthesis chain) changes no
    output; every detector records one launch of each synthesis stage, detector 0 the
    batch's one gather."""
    torch, api, dev = env
    dets, sky = _small_batch(torch, dev)
    b = api.Batch(dets, 80)
    ref = [t.clone() for t in b.run(sky, use_graph=False)]
    views = [b.plan(d) for d in range(len(SMALL))]
    for v in views:
        v.enable_timing(True)
    out = [t.clone() for t in b.run(sky, use_graph=False)]
    torch.cuda.synchronize()
    for d, v in enumerate(views):
        st = v.stage_times()
        v.enable_timing(False)
        for name in ("ring_sums", "theta_upsample", "phi_synthesis", "binning"):
            assert st[name][1] == 1 and st[name][0] >= 0.0, (d, name, st[name])
        assert st["gather"][1] == (1 if d == 0 else 0)
    for x, y in zip(ref, out):
        assert torch.equal(x, y)
    graph = [t.clone() for t in b.run(sky, use_graph=True)]
    torch.cuda.synchronize()
    for x, y in zip(ref, graph):
        assert torch.equal(x, y)


def test_batch_chain_count_leaves_results(env):
    """One to four synthesis chains (SC_PARAM_BATCH_CHAINS): the same kernels on the same data,
    so eager passes and graph replays give the same bits whatever the chain count."""
    torch, api, dev = env
    dets, sky = _small_batch(torch, dev)
    b = api.Batch(dets, 80)
    assert b.get_param("batch_chains") == 4
    ref = [t.clone() for t in b.run(sky, use_graph=False)]
    for nch in (1, 2, 3, 4):
        b.set_param("batch_chains", nch)
        assert b.get_param("batch_chains") == nch
        for g in (False, True, True):
            out = [t.clone() for t in b.run(sky, use_graph=g)]
            torch.cuda.synchronize()
            for x, y in zip(ref, out):
                assert torch.equal(x, y), (nch, g)
    with pytest.raises(api.N.ScError):
        b.set_param("batch_chains", 5)
