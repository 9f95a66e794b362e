"""lmax 1024 support and the mixed-precision form (the precision variant).

* FP64 ring sums at lmax 1024 and 1300 next to the poles (extended-exponent start
  values down to ~1e-2900) against the oracle.
* Mixed precision: the FP64 recursion with the ring contraction on the matrix
  cores (d values and coefficient products rounded to FP32, FP32 products and
  accumulation over 64 steps, then FP64 sums).  Each FP32 rounding is at most
  2^-24 relative; a 64-term FP32 partial sum can lose up to 64 2^-24 = 3.8e-6 of
  the sum of its magnitudes, so the ring sums are held to 4e-6 of the ring's
  largest value, and the TOD to the form's 1e-6 target.
* The precision workload (lmax 1024, kmax 16, 1e8 scan samples) in both the
  mixed and the FP64-recursion forms, against 200 stored oracle samples.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()
    return torch, api, torch.device("cuda", 0)


def _to(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 4e-6)])
def test_ring_sums_start_below_range_then_emerge(env, oracle_lib, prec, tol):
    """lmax 1300: at rings near 22 and 158 degrees the start values of m ~ 430-460
    lie below 2^-600 (e < 0) and the columns grow to ~1e-5 by lmax, so every
    rescaling step is exercised; checked per (k, m) column against the oracle,
    relative to the largest ring sum on the ring."""
    torch, api, dev = env
    L, K = 1300, 2
    a = W.sky_alm(L, 6800)
    b = W.beam_alm(L, K, 6801)
    plan = api.Plan(L, K, prec)
    plan.set_sky_beam(_to(torch, dev, a), _to(torch, dev, b))
    F = plan.debug_stage(0)
    nr = plan.info()["n_rings"]
    js = np.array([nr // 8, nr // 2, 7 * nr // 8])
    th = (js + 0.5) * math.pi / nr
    Fs = F[:, :, torch.as_tensor(js, device=dev)].cpu().numpy()
    ref = np.transpose(oracle_lib.ring_sums(a, b, L, K, th), (0, 2, 1))
    for q in range(len(js)):
        scale = np.max(np.abs(ref[:, :, q]))
        err = np.max(np.abs(Fs[:, :, q] - ref[:, :, q])) / scale
        print("%s ring %d/%d: max error / ring max %.3e" % (prec, js[q], nr, err))
        assert err <= tol, js[q]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 4e-6)])
def test_ring_sums_lmax1024_near_poles(env, oracle_lib, prec, tol):
    torch, api, dev = env
    L, K = 1024, 16
    a = W.sky_alm(L, W.config_seed(3, 1))
    b = W.beam_alm(L, K, W.config_seed(3, 2))
    plan = api.Plan(L, K, prec)
    plan.set_sky_beam(_to(torch, dev, a), _to(torch, dev, b))
    F = plan.debug_stage(0)
    nr = plan.info()["n_rings"]
    js = np.array([0, 3, nr // 2, nr - 1])
    Fs = F[:, :, torch.as_tensor(js, device=dev)].cpu().numpy()
    ref = np.transpose(oracle_lib.ring_sums(a, b, L, K, (js + 0.5) * math.pi / nr), (0, 2, 1))
    for q in range(len(js)):
        err = np.max(np.abs(Fs[:, :, q] - ref[:, :, q])) / np.max(np.abs(ref[:, :, q]))
        print("%s ring %d: max err / max %.3e" % (prec, js[q], err))
        assert err <= tol


@pytest.mark.parametrize("L,K", [(16, 3), (64, 4), (200, 30)])
def test_mixed_ring_sums_small(env, oracle_lib, L, K):
    torch, api, dev = env
    a = W.sky_alm(L, 70 + L)
    b = W.beam_alm(L, K, 80 + L)
    plan = api.Plan(L, K, "mixed")
    plan.set_sky_beam(_to(torch, dev, a), _to(torch, dev, b))
    F = plan.debug_stage(0).cpu().numpy()
    nr = plan.info()["n_rings"]
    ref = np.transpose(oracle_lib.ring_sums(a, b, L, K, (np.arange(nr) + 0.5) * math.pi / nr), (0, 2, 1))
    err = np.max(np.abs(F - ref)) / np.max(np.abs(ref))
    print("mixed ring sums L=%d K=%d: %.3e" % (L, K, err))
    assert err <= 4e-6


@pytest.mark.parametrize("prec", ["mixed", "f64maps_f32gather"])
def test_precision_workload_against_stored_oracle(env, prec):
    """lmax 1024, kmax 16, 1e8 scan samples: 200 stored oracle samples (eight edge
    pointings among them), rel-L2 <= 1e-6 and max|d|/max|c| <= 1e-5."""
    from parity import assert_parity, coef_hash, load_golden, place_golden
    torch, api, dev = env
    (g,) = load_golden("precision-lmax1024-kmax16-scan1e8")
    L, K, n = g["lmax"], g["kmax"], g["n"]
    a = W.sky_alm(L, W.config_seed(3, 1))
    b = W.beam_alm(L, K, W.config_seed(3, 2))
    assert coef_hash(a, b) == g["coef_sha"]
    ptg = W.scan_pointings(n, device=dev)
    it = place_golden(torch, ptg, g)
    plan = api.Plan(L, K, prec)
    tod = plan.convolve(_to(torch, dev, a), _to(torch, dev, b), ptg)
    torch.cuda.synchronize()
    assert_parity(tod[it].double().cpu().numpy(), g["c"], 1e-6, "precision workload %s" % prec)
