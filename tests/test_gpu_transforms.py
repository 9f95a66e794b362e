"""Transform lengths: every radix pass of the LDS FFT and every size class.

The band limits below give theta, upsampled-theta and phi transform lengths
whose radix plans together use every pass radix (2, 3, 4, 5, 6, 8, 9, 10, 12,
15, 16), in the forward (theta analysis) and inverse (upsampling, phi
synthesis) directions, and lmax 1800 needs 7290- and 7500-point transforms
(the 1024-thread class), lmax 2100 8640-point and lmax 2303 (the largest plan) 9216-point
ones (9 points per thread); lmax 256, 512 and 1024 run the compile-time plans of
540/1080, 1080/2160 and 2160/4320 points.  The FP64 form (W = 14) reaches the convolution of
Eq. 2 (Galloway et al. 2022, Sec. 2.1) to ~1e-13, so any wrong twiddle, index
or pass order shows as an O(1) error against the oracle.  The adjoint at the
largest lengths is checked by the dot-product test against its own forward.
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
    api.N.load()
    return torch, api, torch.device("cuda", 0)


def _to(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("L", [6, 10, 13, 15, 24, 32, 40, 64, 100, 256, 512, 1024, 1800, 2100, 2303])
def test_fp64_form_across_transform_lengths(env, oracle_lib, L):
    torch, api, dev = env
    K = min(2, L)
    n = 40 if L > 1000 else 300
    a = W.sky_alm(L, 5000 + L)
    b = W.beam_alm(L, K, 5100 + L)
    p = W.uniform_pointings(n, 5200 + L)
    p[0] = [0.0, 1.0, 2.0]
    p[1] = [math.pi, 0.5, 0.25]
    plan = api.Plan(L, K, "fp64")
    plan.set_sky_beam(_to(torch, dev, a), _to(torch, dev, b))
    tod = plan.interpolate(_to(torch, dev, p)).cpu().numpy()
    ref = oracle_lib.convolve(a, b, L, K, p)
    inf = plan.info()
    assert_parity(tod, ref, 1e-11, "L=%d lengths %d/%d/%d" % (L, inf["n_fft_theta"], inf["n_theta_fine"], inf["n_phi"]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("f64maps_f32gather", 1e-5)])
def test_adjoint_dot_product_largest_lengths(env, prec, tol):
    """<y, A x> = Re sum conj(A^T y) x at lmax 1800 (transforms of 3750, 7500 and 7290 points)."""
    torch, api, dev = env
    L, K, n = 1800, 2, 20000
    a = _to(torch, dev, W.sky_alm(L, 5300))
    b = _to(torch, dev, W.beam_alm(L, K, 5301))
    p = _to(torch, dev, W.uniform_pointings(n, 5302))
    plan = api.Plan(L, K, prec)
    y = torch.randn(n, generator=torch.Generator(device=dev).manual_seed(5303), device=dev,
                    dtype=torch.float64).to(plan.tod_dtype)
    plan.set_sky_beam(a, b)
    tod = plan.interpolate(p)
    g = plan.adjoint(b, p, y)
    lhs = float(torch.dot(tod.double(), y.double()))
    rhs = float(torch.sum(torch.conj(g) * a).real)
    e = abs(lhs - rhs) / abs(lhs)
    print("dot test %s L=%d: %.3e" % (prec, L, e))
    assert e <= tol


def test_adjoint_ring_slabs_lmax_2100(env, oracle_lib):
    """lmax 2100 has 2160 rings, more than one adjoint workgroup holds (2048): the adjoint
    recursion runs in two ring slabs reduced in a fixed order.  Sky and beam gradients
    against the oracle's direct adjoints on a few samples, and the dot-product test."""
    torch, api, dev = env
    from parity import assert_parity
    L, K, n = 2100, 1, 12
    a_np, b_np = W.sky_alm(L, 5400), W.beam_alm(L, K, 5401)
    p_np = W.uniform_pointings(n, 5402)
    p_np[0] = [0.0, 0.3, 1.0]
    y_np = np.random.default_rng(5403).standard_normal(n)
    a, b, p, y = (_to(torch, dev, v) for v in (a_np, b_np, p_np, y_np))
    plan = api.Plan(L, K, "fp64")
    assert plan.info()["n_rings"] > 2048
    plan.set_sky_beam(a, b)
    tod = plan.interpolate(p)
    g = plan.adjoint(b, p, y)
    lhs = float(torch.dot(tod, y))
    rhs = float(torch.sum(torch.conj(g) * a).real)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert_parity(g.cpu().numpy(), oracle_lib.adjoint(b_np, L, K, p_np, y_np), 1e-10, "sky adjoint L=2100")
