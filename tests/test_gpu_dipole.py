"""GPU parity for the orbital dipole / quadrupole response (Galloway et al. 2022, Sec. 3.3).

sc_dipole_response forms the beam moments S, S2 from the l <= 2 beam
coefficients in closed form and evaluates T0 [u.S + q u^T S2 u], u = R^T beta,
per sample.  The reference is the oracle: the moments by quadrature of the
beam field (oracle.brute.beam_moments) with the rotation written out
(oracle.brute.rotation), a relation pinned against the oracle's full
convolution (test_P7_dipole_quadrupole_beam_moments); one test also compares
with that full convolution directly.  Tolerance: 1e-12 of the largest |output|
(FP64 throughout).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

T0, Q = 2.7255, 1.25


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()  # fail loudly if the HIP library is missing
    assert torch.cuda.is_available()
    return torch, api, torch.device("cuda", 0)


def _reference(b, L, K, ptg, beta, spp):
    from oracle.brute import beam_moments, rotation
    S, S2 = beam_moments(b, L, K)
    out = np.empty(ptg.shape[0])
    for s, (th, ph, ps) in enumerate(ptg):
        u = rotation(th, ph, ps).T @ beta[s // spp]
        out[s] = T0 * (u @ S + Q * u @ S2 @ u)
    return out


def _velocities(nper, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nper, 3))
    return 1e-4 * v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.5, 1.5, (nper, 1))


@pytest.mark.parametrize("L,K,kind,n,spp", [(16, 4, "uniform", 3001, 7), (8, 2, "scan", 5000, 1950),
                                            (5, 1, "uniform", 257, 1), (3, 0, "uniform", 100, 100),
                                            (1, 1, "uniform", 64, 5)])
def test_dipole_matches_oracle(env, L, K, kind, n, spp):
    torch, api, dev = env
    b = W.beam_alm(L, K, W.config_seed(60, L))
    ptg = W.scan_pointings(n) if kind == "scan" else W.uniform_pointings(n, W.config_seed(61, n))
    ptg[0] = [0.0, 0.7, 1.1]  # the north pole
    nper = (n + spp - 1) // spp
    beta = _velocities(nper, W.config_seed(62, n))
    got = api.dipole_response(torch.from_numpy(b).to(dev), L, K, torch.from_numpy(ptg).to(dev),
                              torch.from_numpy(beta).to(dev), spp, T0, Q).cpu().numpy()
    ref = _reference(b, L, K, ptg, beta, spp)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("dipole L=%d K=%d %s n=%d: max err %.3e" % (L, K, kind, n, err))
    assert err <= 1e-12


def test_dipole_matches_full_convolution(env, oracle_lib):
    """One velocity for all samples: the response equals the convolution of the
    kinematic sky T0 [beta.n + q (beta.n)^2] (its l <= 2 coefficients) with the beam."""
    torch, api, dev = env
    from oracle.brute import analyse
    L, K, n = 2, 2, 40
    beta = np.array([2e-4, -1e-4, 0.7e-4])
    a = analyse(lambda v: T0 * (beta @ v + Q * (beta @ v) ** 2), L)
    b = W.beam_alm(L, K, W.config_seed(63, 1))
    ptg = W.uniform_pointings(n, W.config_seed(63, 2))
    ref = oracle_lib.convolve(a, b, L, K, ptg)
    got = api.dipole_response(torch.from_numpy(b).to(dev), L, K, torch.from_numpy(ptg).to(dev),
                              torch.from_numpy(beta[None, :]).to(dev), n, T0, Q).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dipole_argument_errors(env):
    torch, api, dev = env
    from paper_2201_03478_amd import _native as N
    lib = N.load()
    b = torch.zeros(W.n_alm(4, 2), dtype=torch.complex128, device=dev)
    ptg = torch.zeros((10, 3), dtype=torch.float64, device=dev)
    beta = torch.zeros((10, 3), dtype=torch.float64, device=dev)
    out = torch.zeros(10, dtype=torch.float64, device=dev)
    # n = 0 is a no-op; host memory and bad sizes are rejected before any launch
    assert lib.sc_dipole_response(b.data_ptr(), 4, 2, ptg.data_ptr(), 0, beta.data_ptr(), 1, T0, Q,
                                  out.data_ptr(), None) == N.SC_OK
    host = np.zeros(30)
    assert lib.sc_dipole_response(b.data_ptr(), 4, 2, host.ctypes.data, 10, beta.data_ptr(), 1, T0, Q,
                                  out.data_ptr(), None) == N.SC_EINVAL
    assert lib.sc_dipole_response(b.data_ptr(), 4, 2, ptg.data_ptr(), 10, beta.data_ptr(), 0, T0, Q,
                                  out.data_ptr(), None) == N.SC_EINVAL
    assert lib.sc_dipole_response(b.data_ptr(), 4, 5, ptg.data_ptr(), 10, beta.data_ptr(), 1, T0, Q,
                                  out.data_ptr(), None) == N.SC_EINVAL
