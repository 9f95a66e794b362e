"""sc_interpolate_noalloc (binning workspace in the library's fixed per-GPU array)
against sc_interpolate (plan workspace), through the C ABI.

Both run the same binning and gather kernels; the no-allocation form bins in
passes of what its array holds, and every sample's arithmetic is independent of
the pass and of the other samples of its work item, so the two agree bit for bit
(the parity bar of the FP32 and FP64 forms is met a fortiori).
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()
    return torch, api, torch.device("cuda", 0)


def _noalloc(api, plan, ptg, out):
    rc = api.N.load().sc_interpolate_noalloc(plan._p, ctypes.c_void_p(ptg.data_ptr()), ptg.shape[0],
                                             ctypes.c_void_p(out.data_ptr()))
    api.N.check(rc, "sc_interpolate_noalloc")
    return out


@pytest.mark.parametrize("prec", ["f64maps_f32gather", "fp64"])
def test_noalloc_matches_interpolate_twice(env, prec):
    """lmax 512, kmax 100 with 1e7 scan samples (three passes through the array), then a
    smaller, ragged call of 123,457 samples on the same plan."""
    torch, api, dev = env
    L, K = 512, 100
    a = torch.from_numpy(W.sky_alm(L, W.config_seed(2, 1))).to(dev)
    b = torch.from_numpy(W.beam_alm(L, K, W.config_seed(2, 2))).to(dev)
    plan = api.Plan(L, K, prec, kernel_width=8)
    plan.set_sky_beam(a, b)
    for n, start in ((10_000_000, 0), (123_457, 3_000_001)):
        ptg = W.scan_pointings(n, start=start, device=dev)
        ref = plan.interpolate(ptg).clone()
        out = torch.full_like(ref, float("nan"))
        _noalloc(api, plan, ptg, out)
        torch.cuda.synchronize()
        sel = torch.arange(0, n, max(1, n // 4000), device=dev)
        assert_parity(out[sel].double().cpu().numpy(), ref[sel].double().cpu().numpy(),
                      1e-6 if prec != "fp64" else 1e-12, "noalloc %s n=%d" % (prec, n))
        assert torch.equal(out, ref), (prec, n)


def test_noalloc_rejects_a_grid_above_its_array(env):
    torch, api, dev = env
    L, K = 2000, 0
    plan = api.Plan(L, K, "f64maps_f32gather")
    a = torch.from_numpy(W.sky_alm(L, 9)).to(dev)
    b = torch.from_numpy(W.beam_alm(L, K, 10)).to(dev)
    plan.set_sky_beam(a, b)
    ptg = W.scan_pointings(1000, device=dev)
    out = torch.zeros(1000, dtype=torch.float32, device=dev)
    rc = api.N.load().sc_interpolate_noalloc(plan._p, ctypes.c_void_p(ptg.data_ptr()), 1000,
                                             ctypes.c_void_p(out.data_ptr()))
    assert rc == api.N.SC_EINVAL
    assert b"scratch" in api.N.load().sc_last_error()
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was launched
