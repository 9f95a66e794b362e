"""Validation mode (SC_PARAM_VALIDATE): NaN and infinite inputs are refused with
SC_EINVAL naming the input, before any launch; with the mode off (the default)
nothing is inspected and a NaN angle is read as 0."""
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


@pytest.mark.parametrize("prec", ["f64maps_f32gather", "fp64"])
def test_validation_refuses_nonfinite_inputs(env, prec):
    torch, api, dev = env
    L, K, n = 32, 4, 700
    a, b = _to(torch, dev, W.sky_alm(L, 7100)), _to(torch, dev, W.beam_alm(L, K, 7101))
    ptg = _to(torch, dev, W.uniform_pointings(n, 7102))
    ref_plan = api.Plan(L, K, prec)
    ref = ref_plan.convolve(a, b, ptg).clone()
    plan = api.Plan(L, K, prec)
    plan.set_param("validate", 1)
    assert plan.get_param("validate") == 1
    out = plan.convolve(a, b, ptg)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)  # clean inputs: the same launches, the same result

    bad = ptg.clone()
    bad[17, 1] = float("nan")
    bad[40, 2] = float("inf")
    with pytest.raises(api.N.ScError, match="ptg holds 2 NaN or infinite"):
        plan.convolve(a, b, bad)
    with pytest.raises(api.N.ScError, match="ptg holds 2"):
        plan.interpolate(bad)
    a_bad = a.clone()
    a_bad[5] = complex(float("inf"), 0.0)
    with pytest.raises(api.N.ScError, match="alm holds 1"):
        plan.set_sky_beam(a_bad, b)
    b_bad = b.clone()
    b_bad[3] = complex(0.0, float("nan"))
    with pytest.raises(api.N.ScError, match="blm holds 1"):
        plan.convolve(a, b_bad, ptg)
    y = torch.randn(n, device=dev).to(plan.tod_dtype)
    y[9] = float("nan")
    with pytest.raises(api.N.ScError, match="tod_grad holds 1"):
        plan.adjoint(b, ptg, y)
    # the plan still works after the refusals
    out2 = plan.convolve(a, b, ptg)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)


def test_default_mode_reads_nan_angle_as_zero(env):
    torch, api, dev = env
    L, K, n = 24, 3, 64
    a, b = _to(torch, dev, W.sky_alm(L, 7200)), _to(torch, dev, W.beam_alm(L, K, 7201))
    p = W.uniform_pointings(n, 7202)
    p_nan, p_zero = p.copy(), p.copy()
    p_nan[5, 1] = math.nan
    p_zero[5, 1] = 0.0
    plan = api.Plan(L, K, "fp64")
    plan.set_sky_beam(a, b)
    t_nan = plan.interpolate(_to(torch, dev, p_nan)).cpu().numpy()
    t_zero = plan.interpolate(_to(torch, dev, p_zero)).cpu().numpy()
    assert np.array_equal(t_nan, t_zero)
