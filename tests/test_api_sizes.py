"""CPU-side argument checks of the Python binding.

The C ABI takes plain pointers, so it cannot see tensor sizes: the binding must
reject a mis-sized tensor before any pointer reaches the library (a short buffer
would be read or written past its end on the device).  These checks run before
any device access, so they are exercised here with CPU tensors.
"""
import ctypes

import pytest
import torch

from paper_2201_03478_amd import api


def _c(n):
    return torch.zeros(n, dtype=torch.complex128)


def _p(n):
    return torch.zeros((n, 3), dtype=torch.float64)


L, K = 16, 4
NA, NB = api.n_alm(L), api.n_alm(L, K)


@pytest.mark.parametrize("args", [
    dict(alm=_c(NA - 1)), dict(alm=_c(NA + 1)), dict(blm=_c(NB - 1)), dict(blm=_c(NA)),
    dict(ptg=torch.zeros(30, dtype=torch.float64)), dict(ptg=torch.zeros((10, 2), dtype=torch.float64)),
    dict(ptg=torch.zeros((10, 3, 1), dtype=torch.float64)), dict(out=torch.zeros(9, dtype=torch.float32)),
    dict(out=torch.zeros(11, dtype=torch.float32)), dict(kmax=L + 1), dict(kmax=-1),
])
def test_one_shot_convolve_rejects_bad_sizes(args):
    kw = dict(alm=_c(NA), blm=_c(NB), lmax=L, kmax=K, ptg=_p(10), out=None)
    kw.update(args)
    with pytest.raises(ValueError):
        api.convolve(kw["alm"], kw["blm"], kw["lmax"], kw["kmax"], kw["ptg"], out=kw["out"])


def test_one_shot_convolve_good_sizes_reach_the_device_check():
    """With every size right, the next check is that the tensors live on the GPU."""
    with pytest.raises(TypeError):
        api.convolve(_c(NA), _c(NB), L, K, _p(10))


def _plan_without_device():
    # a Plan object whose handle is NULL: only the Python-side checks can run
    return api.Plan(L, K, "f64maps_f32gather", _handle=ctypes.c_void_p())


@pytest.mark.parametrize("args", [
    dict(blm=_c(NB + 1)), dict(ptg=torch.zeros((10, 4), dtype=torch.float64)),
    dict(tod_grad=torch.zeros(11, dtype=torch.float32)), dict(out=_c(NA - 1)), dict(out=_c(NB)),
])
def test_plan_adjoint_rejects_bad_sizes(args):
    kw = dict(blm=_c(NB), ptg=_p(10), tod_grad=torch.zeros(10, dtype=torch.float32), out=None)
    kw.update(args)
    with pytest.raises(ValueError):
        _plan_without_device().adjoint(kw["blm"], kw["ptg"], kw["tod_grad"], out=kw["out"])


@pytest.mark.parametrize("method", ["interpolate", "interpolate_psi"])
@pytest.mark.parametrize("ptg,out", [
    (torch.zeros((10, 2), dtype=torch.float64), None),
    (_p(10), torch.zeros(12, dtype=torch.float32)),
])
def test_plan_interpolate_rejects_bad_sizes(method, ptg, out):
    with pytest.raises(ValueError):
        getattr(_plan_without_device(), method)(ptg, out=out)


@pytest.mark.parametrize("args", [
    dict(blm=_c(NB - 1)), dict(ptg=torch.zeros((5, 2), dtype=torch.float64)),
    dict(beta=torch.zeros((1, 3), dtype=torch.float64)), dict(out=torch.zeros(4, dtype=torch.float64)),
    dict(spp=0),
])
def test_dipole_rejects_bad_sizes(args):
    kw = dict(blm=_c(NB), ptg=_p(5), beta=torch.zeros((3, 3), dtype=torch.float64), spp=2, out=None)
    kw.update(args)
    with pytest.raises(ValueError):
        api.dipole_response(kw["blm"], L, K, kw["ptg"], kw["beta"], kw["spp"], 2.7, 1.25, out=kw["out"])
