"""GPU parity for the psi cube (the second step of the two-step algorithm, Galloway et al.
2022, Sec. 2.1): the cube c(theta, phi, psi) on an oversampled psi grid, then
three-dimensional interpolation with the exponential-of-semicircle kernel.

The method approximates the plain sum of Eq. 2, so the reference is the oracle's direct
sum on the same seeded inputs.  The cube adds the kernel's error along psi to the two
in (theta, phi); with the same width and twofold oversampling that error is of the same
order, so the bars are those of the two-dimensional gather:
  * FP64 plan, W = 14: rel-L2 <= 1e-12 (kernel error ~4e-14 per axis + rounding);
  * FP32 plan, W = 8: rel-L2 <= 1e-6 (kernel error ~3e-8 per axis, FP32 map and cube
    rounding ~1e-7).
At the lmax 512 / kmax 100 size the cube path is compared with the exact k-sum path on
every sample (both approximate the same sum) and with the oracle on a sample.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()  # fail loudly if the HIP library is missing
    assert torch.cuda.is_available()
    return torch, api, torch.device("cuda", 0)


def _rel_l2(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def _setup(api, torch, dev, L, K, prec, seed, width=0):
    a = W.sky_alm(L, W.config_seed(seed, 1))
    b = W.beam_alm(L, K, W.config_seed(seed, 2))
    plan = api.Plan(L, K, prec, kernel_width=width)
    plan.set_sky_beam(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    return a, b, plan


def _edge_pointings(n, seed):
    """Uniform pointings with poles, psi at and beyond the period and negative angles."""
    p = W.uniform_pointings(n, seed)
    p[0] = [0.0, 0.3, 0.0]
    p[1] = [math.pi, 1.0, 2 * math.pi]
    p[2] = [1.0, -0.5, -2.0]
    p[3] = [2.0, 7.0, 13.0]
    p[4] = [0.5, 2 * math.pi - 1e-13, 2 * math.pi - 1e-13]
    return p


@pytest.mark.parametrize("L,K,prec,n,bar", [(32, 4, "fp64", 1500, 1e-12), (20, 20, "fp64", 700, 1e-12),
                                            (8, 0, "fp64", 300, 1e-12), (64, 8, "f64maps_f32gather", 3000, 1e-6),
                                            (40, 17, "f64maps_f32gather", 2000, 1e-6),
                                            (1, 1, "f64maps_f32gather", 200, 1e-6),
                                            (40, 17, "fp64", 800, 1e-12), (64, 32, "fp64", 800, 1e-12),
                                            (64, 32, "f64maps_f32gather", 2000, 1e-6)])
def test_psi_cube_matches_oracle(env, oracle_lib, L, K, prec, n, bar):
    """Default psi grids: 30, 36, 90 points (runtime-planned transform, one per wave), 72 and 135
    (compile-time plans, four and two transforms per wave), 16."""
    torch, api, dev = env
    a, b, plan = _setup(api, torch, dev, L, K, prec, 70 + L + K)
    ptg = _edge_pointings(n, W.config_seed(71, n))
    plan.build_psi_cube()
    got = plan.interpolate_psi(torch.from_numpy(ptg).to(dev)).double().cpu().numpy()
    ref = oracle_lib.convolve(a, b, L, K, ptg)
    assert_parity(got, ref, bar, "psi cube L=%d K=%d %s n=%d" % (L, K, prec, n))


def test_psi_cube_grid_sizes_and_rebuild(env, oracle_lib):
    """Explicit psi grids (larger than the default, an odd size) give the same result; the
    plan reallocates the cube when the size changes and keeps it when it does not."""
    torch, api, dev = env
    L, K = 24, 6
    a, b, plan = _setup(api, torch, dev, L, K, "fp64", 72)
    ptg = _edge_pointings(800, W.config_seed(72, 3))
    ref = oracle_lib.convolve(a, b, L, K, ptg)
    pt = torch.from_numpy(ptg).to(dev)
    for npsi in (0, 45, 64, 75, 0):
        plan.build_psi_cube(npsi)
        got = plan.interpolate_psi(pt).cpu().numpy()
        assert_parity(got, ref, 1e-12, "psi cube npsi=%d" % npsi)


def test_psi_cube_state_and_argument_errors(env):
    torch, api, dev = env
    from paper_2201_03478_amd import _native as N
    lib = N.load()
    L, K = 16, 3
    a, b, plan = _setup(api, torch, dev, L, K, "fp64", 73)
    ptg = torch.from_numpy(W.uniform_pointings(10, 5)).to(dev)
    out = torch.zeros(10, dtype=torch.float64, device=dev)
    # no cube yet
    assert lib.sc_interpolate_psi(plan._p, ptg.data_ptr(), 10, out.data_ptr()) == N.SC_ESTATE
    # sizes: below 2 (2 kmax + 1) = 14 or 2 W = 28, not 2,3,5-smooth, above 512
    for bad in (26, 14, 49, 77, 540, -3):
        assert lib.sc_plan_build_psi_cube(plan._p, bad) == N.SC_EINVAL, bad
    assert lib.sc_plan_build_psi_cube(plan._p, 0) == N.SC_OK
    assert lib.sc_interpolate_psi(plan._p, ptg.data_ptr(), 0, out.data_ptr()) == N.SC_OK
    host = np.zeros(30)
    assert lib.sc_interpolate_psi(plan._p, host.ctypes.data, 10, out.data_ptr()) == N.SC_EINVAL
    assert lib.sc_interpolate_psi(plan._p, ptg.data_ptr(), 10, out.data_ptr()) == N.SC_OK
    # new maps invalidate the cube
    plan.set_sky_beam(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    assert lib.sc_interpolate_psi(plan._p, ptg.data_ptr(), 10, out.data_ptr()) == N.SC_ESTATE
    # a plan without maps
    fresh = api.Plan(L, K, "fp64")
    assert lib.sc_plan_build_psi_cube(fresh._p, 0) == N.SC_ESTATE


def test_psi_cube_full_size(env, oracle_lib):
    """lmax 512, kmax 100, 1e7 scan samples: the cube path against the exact k-sum path on
    every sample, and against the oracle on 16 samples."""
    torch, api, dev = env
    L, K, n = 512, 100, 10_000_000
    a, b, plan = _setup(api, torch, dev, L, K, "f64maps_f32gather", 2)
    ptg = torch.from_numpy(W.scan_pointings(n)).to(dev)
    plan.build_psi_cube()
    got = plan.interpolate_psi(ptg)
    exact = plan.interpolate(ptg)
    d = float(torch.linalg.vector_norm((got - exact).double()) / torch.linalg.vector_norm(exact.double()))
    print("psi cube full size: rel-L2 vs k-sum path %.3e" % d)
    assert d <= 1e-6
    d_max = float((got - exact).abs().max() / exact.abs().max())
    print("psi cube full size: max|d|/max|c| vs k-sum path %.3e" % d_max)
    assert d_max <= 1e-5
    from parity import load_golden
    (g,) = load_golden("sidelobe-lmax512-kmax100-scan1e7")
    it = torch.as_tensor(g["idx"][9:], device=dev)  # the scan's own samples (not the edge pointings)
    assert_parity(got[it].double().cpu().numpy(), g["c"][9:], 1e-6, "psi cube full size vs stored oracle")


def _with_env(env, fn):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("passmax", [None, "70000"])
def test_psi_binned_order_is_bit_identical(env, oracle_lib, passmax):
    """The FP32 cube gather takes samples in anchor order (the binning); each sample's arithmetic
    is that of the per-sample order, so the two agree bit for bit, also over several binning passes."""
    torch, api, dev = env
    L, K, n = 96, 12, 200_001
    a = W.sky_alm(L, W.config_seed(74, 1))
    b = W.beam_alm(L, K, W.config_seed(74, 2))
    ptg = torch.from_numpy(np.concatenate([W.scan_pointings(n - 5000), _edge_pointings(5000, 75)])).to(dev)

    def run():
        plan = api.Plan(L, K, "f64maps_f32gather")
        plan.set_sky_beam(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
        plan.build_psi_cube()
        out = plan.interpolate_psi(ptg)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    env_b = {"SC_BIN_PASS_MAX": passmax} if passmax else {}
    binned = _with_env(env_b, run) if env_b else run()
    direct = _with_env({"SC_GATHER_PATH": "direct"}, run)
    assert np.array_equal(binned, direct)
    idx = np.linspace(0, n - 1, 64).astype(np.int64)
    ref = oracle_lib.convolve(a, b, L, K, ptg[torch.as_tensor(idx, device=dev)].cpu().numpy())
    assert_parity(binned[idx].astype(np.float64), ref, 1e-6, "psi binned order")


@pytest.mark.parametrize("width", [4, 6, 10, 12, 16])
def test_psi_fp32_other_widths(env, oracle_lib, width):
    """FP32 cube at other kernel widths (2 to 5 quads per psi run, unbinned order): its error
    against the oracle stays at the level of the two-dimensional gather of the same width, the
    psi axis adding an error of the same kind as theta and phi."""
    torch, api, dev = env
    L, K, n = 48, 10, 3000
    a, b, plan = _setup(api, torch, dev, L, K, "f64maps_f32gather", 76, width=width)
    ptg = _edge_pointings(n, W.config_seed(77, width))
    pt = torch.from_numpy(ptg).to(dev)
    plan.build_psi_cube()
    got = plan.interpolate_psi(pt).double().cpu().numpy()
    two_d = plan.interpolate(pt).double().cpu().numpy()
    ref = oracle_lib.convolve(a, b, L, K, ptg)
    from parity import errors
    (e3, m3), (e2, m2) = errors(got, ref), errors(two_d, ref)
    print("psi cube FP32 W=%d: rel-L2 %.3e max %.3e (2-D gather %.3e, %.3e)" % (width, e3, m3, e2, m2))
    assert e3 <= 3.0 * e2 + 1e-6
    assert m3 <= 3.0 * m2 + 1e-5
