"""Synthetic sky, beam, pointing and residual generators.

The paper's own inputs (LFI sidelobe models stored with lmax = 512 and
mmax = 100, the Commander sky and the Planck pointing; Galloway et al. 2022,
Secs. 2.2 and 3) are not available, so these seeded stand-ins take their shapes:

* sky a_lm: a_00 = 0 and, for l >= 1, Gaussian with C_l = 1/(l(l+1)); a_l0 real.
* beam b_lk, 0 <= k <= min(l, kmax): a complex Gaussian (unit variance, real at
  k = 0) times either a Gaussian-beam window exp(-l(l+1) sigma^2 / 2), the
  sidelobe-like envelope (1+k)^-1.5 exp(-l/200), or (1+k)^-1.5 alone (flat in l,
  to exercise every multipole of a high band limit).
* pointings: uniform on the sphere with uniform psi, or a synthetic scan: the
  boresight sweeps a circle of 85 deg opening angle around a spin axis in the
  ecliptic plane at 1 rpm, sampled at 32.5 Hz, with the spin axis advancing
  1 deg/day and psi tied to the scan direction (plus a per-detector offset).

Layout: complex128 m-major triangular arrays, index(l, m) = m (2 lmax + 1 - m)/2 + l;
pointings float64 [n, 3] = (theta, phi, psi).
"""
from __future__ import annotations

import math

import numpy as np

# Workloads by name; "seed" is the namespace of their seeds (config_seed).
CONFIGS = {
    "fp64-tiny": dict(seed=1, lmax=64, kmax=4, n=100_000, beam="gauss", pointing="uniform"),
    "sidelobe-lmax512-kmax100": dict(seed=2, lmax=512, kmax=100, n=10_000_000, beam="sidelobe",
                                     pointing="scan"),
    "precision-lmax1024-kmax16": dict(seed=3, lmax=1024, kmax=16, n=100_000_000, beam="sidelobe",
                                      pointing="scan"),
    "batched-12det": dict(seed=4, lmax=1024, kmax=100, n=40_000_000, beam="sidelobe", pointing="scan"),
    "adjoint-lmax512-kmax32": dict(seed=5, lmax=512, kmax=32, n=100_000_000, beam="sidelobe",
                                   pointing="scan"),
}

# Batched workload: per-detector (lmax, kmax, n); detector d starts at t0 = d * 1000 s
# with psi offset d * pi / 12 and its own beam seed.
DETECTORS = [
    (1024, 100, 10_000_000), (512, 100, 8_000_000), (256, 100, 6_000_000),
    (1024, 32, 5_000_000), (512, 32, 4_000_000), (256, 32, 3_000_000),
    (1024, 8, 2_000_000), (512, 8, 1_000_000), (256, 8, 500_000),
    (512, 100, 300_000), (1024, 32, 100_000), (256, 8, 100_000),
]

ROLE_SKY, ROLE_BEAM, ROLE_PTG, ROLE_Y, ROLE_FD, ROLE_SUB = 1, 2, 3, 4, 5, 6


def config_seed(config: int, role: int) -> int:
    return 1000 * config + role


def n_alm(lmax: int, mmax: int | None = None) -> int:
    mmax = lmax if mmax is None else mmax
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def _lm_arrays(lmax: int, mmax: int):
    ls, ms = [], []
    for m in range(mmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def sky_alm(lmax: int, seed: int) -> np.ndarray:
    """a_00 = 0; a_l0 ~ N(0, C_l) real; Re, Im a_lm ~ N(0, C_l / 2) for m > 0; C_l = 1/(l(l+1))."""
    rng = np.random.default_rng(seed)
    l, m = _lm_arrays(lmax, lmax)
    cl = np.zeros(l.shape)
    cl[l > 0] = 1.0 / (l[l > 0] * (l[l > 0] + 1.0))
    re = rng.standard_normal(l.size)
    im = rng.standard_normal(l.size)
    a = np.where(m == 0, np.sqrt(cl) * re, np.sqrt(cl / 2) * (re + 1j * im))
    return a.astype(np.complex128)


def beam_alm(lmax: int, kmax: int, seed: int, kind: str = "sidelobe",
             sigma: float = math.radians(5.0)) -> np.ndarray:
    """b_lk = g_lk * envelope; g complex Gaussian of unit variance, real at k = 0."""
    rng = np.random.default_rng(seed)
    l, k = _lm_arrays(lmax, kmax)
    re = rng.standard_normal(l.size)
    im = rng.standard_normal(l.size)
    g = np.where(k == 0, re + 0j, (re + 1j * im) / np.sqrt(2.0))
    if kind == "gauss":
        env = np.exp(-l * (l + 1.0) * sigma * sigma / 2.0)
    elif kind == "sidelobe":
        env = (1.0 + k) ** -1.5 * np.exp(-l / 200.0)
    elif kind == "flat":  # no decay in l: every multipole up to lmax carries weight
        env = (1.0 + k) ** -1.5 + 0.0 * l
    else:
        raise ValueError(kind)
    return (g * env).astype(np.complex128)


def truncate_alm(alm: np.ndarray, lmax_in: int, lmax_out: int, mmax_out: int | None = None) -> np.ndarray:
    """Keep l <= lmax_out (and m <= mmax_out) of an lmax_in array, in the lmax_out layout."""
    mmax_out = lmax_out if mmax_out is None else mmax_out
    out = np.zeros(n_alm(lmax_out, mmax_out), dtype=alm.dtype)
    for m in range(mmax_out + 1):
        src = m * (2 * lmax_in + 1 - m) // 2
        dst = m * (2 * lmax_out + 1 - m) // 2
        out[dst + m: dst + lmax_out + 1] = alm[src + m: src + lmax_out + 1]
    return out


def uniform_pointings(n: int, seed: int) -> np.ndarray:
    """theta = arccos U(-1, 1), phi ~ U[0, 2 pi), psi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    p = np.empty((n, 3))
    p[:, 0] = np.arccos(rng.uniform(-1.0, 1.0, n))
    p[:, 1] = rng.uniform(0.0, 2 * np.pi, n)
    p[:, 2] = rng.uniform(0.0, 2 * np.pi, n)
    return p


def scan_pointings(n: int, start: int = 0, t0: float = 0.0, psi0: float = 0.0,
                   device=None, chunk: int = 1 << 22):
    """Synthetic scan, samples start .. start + n - 1, as float64 [n, 3].

    Spin axis s = (cos lam, sin lam, 0), lam = 1 deg/day * t; spin phase
    w = 2 pi t / 60 s; boresight n = cos(85 deg) s + sin(85 deg)(cos w z + sin w (z x s));
    psi = atan2(v . e_phi, v . e_theta) + psi0 with v = dn/dt.
    With ``device`` set (a torch device) the result is a torch tensor computed there.
    """
    if device is not None:
        import torch
        out = torch.empty((n, 3), dtype=torch.float64, device=device)
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            i = torch.arange(start + s, start + e, dtype=torch.float64, device=device)
            out[s:e] = _scan_block(torch, i, t0, psi0)
        return out
    out = np.empty((n, 3))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i = np.arange(start + s, start + e, dtype=np.float64)
        out[s:e] = _scan_block(np, i, t0, psi0)
    return out


def _scan_block(xp, i, t0, psi0):
    fs = 32.5
    alpha = math.radians(85.0)
    lam_rate = math.radians(1.0) / 86400.0
    w_rate = 2.0 * math.pi / 60.0
    t = t0 + i / fs
    lam = lam_rate * t
    w = w_rate * t
    cl, sl = xp.cos(lam), xp.sin(lam)
    cw, sw = xp.cos(w), xp.sin(w)
    ca, sa = math.cos(alpha), math.sin(alpha)
    # z x s = (-sin lam, cos lam, 0)
    nx = ca * cl + sa * sw * (-sl)
    ny = ca * sl + sa * sw * cl
    nz = sa * cw
    # analytic derivative
    dsx, dsy = -lam_rate * sl, lam_rate * cl
    dzsx, dzsy = -lam_rate * cl, -lam_rate * sl
    vx = ca * dsx + sa * (w_rate * cw * (-sl) + sw * dzsx)
    vy = ca * dsy + sa * (w_rate * cw * cl + sw * dzsy)
    vz = -sa * w_rate * sw
    theta = xp.arccos(xp.clip(nz, -1.0, 1.0))
    phi = xp.remainder(xp.arctan2(ny, nx), 2.0 * math.pi)
    ct, st = xp.cos(theta), xp.sin(theta)
    cp, sp = xp.cos(phi), xp.sin(phi)
    v_th = vx * ct * cp + vy * ct * sp - vz * st
    v_ph = -vx * sp + vy * cp
    psi = xp.remainder(xp.arctan2(v_ph, v_th) + psi0, 2.0 * math.pi)
    return xp.stack([theta, phi, psi], axis=1) if xp is np else xp.stack([theta, phi, psi], dim=1)


def residual(n: int, seed: int) -> np.ndarray:
    """TOD residual y ~ N(0, 1) as float32."""
    return np.random.default_rng(seed).standard_normal(n, dtype=np.float32)
