"""Band limits beyond one workgroup's transforms: lmax 4096 and 8192 (the range of
the runtime comparison of Galloway et al. 2022, Sec. 2.2, Fig. 2).

Above lmax 2303 the theta and phi transforms (up to 34,560 points) run as several
LDS transforms each (k_fft_big.hip), and the adjoint recursion splits each
column's rings into slabs.  Checked against the CPU oracle: FP64 ring sums next
to the poles (start values far below the FP64 range), the FP64 form end to end
(W = 14, <= 1e-11), the FP32-gather form (<= 1e-6), and both adjoints (dot test
and the oracle's direct adjoint).  Samples include both poles, and the beams do
not decay in l, so every multipole up to lmax carries weight.
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


def _pointings(n, seed):
    p = W.uniform_pointings(n, seed)
    p[0] = [0.0, 0.4, 1.3]
    p[1] = [math.pi, 2.2, 0.1]
    p[2] = [1e-7, 6.2831853, 3.0]
    p[3] = [math.pi / 2, 0.0, 0.0]
    return p


CASES = [(4096, 4), (8192, 2)]


@pytest.mark.parametrize("L,K", CASES)
def test_highl_ring_sums_near_poles(env, oracle_lib, L, K):
    torch, api, dev = env
    a_np, b_np = W.sky_alm(L, 9000 + K), W.beam_alm(L, K, 9100 + K, kind="flat")
    plan = api.Plan(L, K, "fp64")
    plan.set_sky_beam(_to(torch, dev, a_np), _to(torch, dev, b_np))
    nr = plan.info()["n_rings"]
    js = np.array([0, 2, nr // 5, nr // 2, nr - 1])
    F = plan.debug_stage(0)[:, :, torch.as_tensor(js, device=dev)].cpu().numpy()
    ref = np.transpose(oracle_lib.ring_sums(a_np, b_np, L, K, (js + 0.5) * math.pi / nr), (0, 2, 1))
    for q in range(len(js)):
        err = np.max(np.abs(F[:, :, q] - ref[:, :, q])) / np.max(np.abs(ref[:, :, q]))
        print("L=%d ring %d/%d: max err / ring max %.3e" % (L, js[q], nr, err))
        assert err <= 1e-11


@pytest.mark.parametrize("L,K", CASES)
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-11), ("f64maps_f32gather", 1e-6)])
def test_highl_end_to_end(env, oracle_lib, L, K, prec, bar):
    torch, api, dev = env
    a_np, b_np = W.sky_alm(L, 9200 + K), W.beam_alm(L, K, 9300 + K, kind="flat")
    p_np = _pointings(24, 9400 + L)
    plan = api.Plan(L, K, prec)
    inf = plan.info()
    assert inf["n_phi"] > 9216  # the split transforms run
    tod = plan.convolve(_to(torch, dev, a_np), _to(torch, dev, b_np), _to(torch, dev, p_np))
    torch.cuda.synchronize()
    ref = oracle_lib.convolve(a_np, b_np, L, K, p_np)
    assert_parity(tod.double().cpu().numpy(), ref, bar, "L=%d K=%d %s (lengths %d/%d/%d)"
                  % (L, K, prec, inf["n_fft_theta"], inf["n_theta_fine"], inf["n_phi"]))


@pytest.mark.parametrize("L,K", CASES)
def test_highl_adjoints(env, oracle_lib, L, K):
    """Sky and beam gradients (FP64): dot-product identities against the forward path and the
    oracle's direct sky adjoint."""
    torch, api, dev = env
    a_np, b_np = W.sky_alm(L, 9500 + K), W.beam_alm(L, K, 9600 + K, kind="flat")
    b_np[:L + 1] = b_np[:L + 1].real
    n = 8
    p_np = _pointings(n, 9700 + L)
    y_np = np.random.default_rng(9800 + L).standard_normal(n)
    a, b, p, y = (_to(torch, dev, v) for v in (a_np, b_np, p_np, y_np))
    plan = api.Plan(L, K, "fp64")
    plan.set_sky_beam(a, b)
    lhs = float(torch.dot(plan.interpolate(p), y))
    g = plan.adjoint(b, p, y)
    rhs = float(torch.sum(torch.conj(g) * a).real)
    print("L=%d sky dot test %.3e" % (L, abs(lhs - rhs) / abs(lhs)))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    h = plan.adjoint_beam(a, p, y)
    rhs_b = float(torch.sum(torch.conj(h) * b).real)
    print("L=%d beam dot test %.3e" % (L, abs(lhs - rhs_b) / abs(lhs)))
    assert abs(lhs - rhs_b) <= 1e-11 * abs(lhs)
    assert_parity(g.cpu().numpy(), oracle_lib.adjoint(b_np, L, K, p_np, y_np), 1e-10, "sky adjoint L=%d" % L)
