"""Brute-force checks for the oracle (test infrastructure only).

Independent routes to the quantities the C oracle computes, used to pin it:

* ``wigner_d_explicit``: Wigner's explicit finite sum for d^l_{mk}(theta) in
  arbitrary precision (mpmath), the textbook definition of the small d-matrix.
* ``conv_quadrature``: the convolution integral of Galloway et al. (2022),
  Sec. 2.1, Eq. 1, evaluated in pixel space: the beam, defined pointing at the
  north pole, is rotated by R = R_z(phi) R_y(theta) R_z(psi) and integrated
  against the sky with a Gauss-Legendre x uniform grid that is exact for the
  band limit.  Spherical harmonics come from ``scipy.special.sph_harm_y``.
* ``beam_moments``: the first and second moments S_i and S_ij of the beam
  (Sec. 3.3, the precomputed geometric factors of the dipole/quadrupole
  shortcut), by the same quadrature.
* ``analyse``: a_lm of a pixel-space function by exact quadrature.

None of this uses a Wigner-d recursion.
"""
from __future__ import annotations

import mpmath
import numpy as np
from scipy.special import sph_harm_y

from . import alm_index, n_alm


def wigner_d_explicit(l: int, m: int, k: int, theta, dps: int = 40):
    """d^l_{mk}(theta) from Wigner's explicit sum, evaluated with mpmath."""
    with mpmath.workdps(dps):
        th = mpmath.mpf(theta)
        c = mpmath.cos(th / 2)
        s = mpmath.sin(th / 2)
        f = mpmath.factorial
        pref = mpmath.sqrt(f(l + m) * f(l - m) * f(l + k) * f(l - k))
        tot = mpmath.mpf(0)
        for q in range(max(0, k - m), min(l + k, l - m) + 1):
            den = f(l + k - q) * f(q) * f(m - k + q) * f(l - m - q)
            sgn = -1 if (m - k + q) % 2 else 1
            tot += sgn * c ** (2 * l + k - m - 2 * q) * s ** (m - k + 2 * q) / den
        return pref * tot


def field_values(coefs, lmax: int, mmax: int, theta, phi) -> np.ndarray:
    """Real field sum_{l, |m| <= min(l, mmax)} a_lm Y_lm(theta, phi) from the stored m >= 0 half."""
    coefs = np.asarray(coefs, dtype=np.complex128)
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    out = np.zeros(np.broadcast(theta, phi).shape)
    for m in range(mmax + 1):
        for l in range(m, lmax + 1):
            a = coefs[alm_index(lmax, l, m)]
            y = sph_harm_y(l, m, theta, phi)
            if m == 0:
                out += a.real * y.real
            else:
                # a_lm Y_lm + a_{l,-m} Y_{l,-m} = 2 Re(a_lm Y_lm) for a real field
                out += 2.0 * (a * y).real
    return out


def gl_sphere_grid(nth: int, nph: int):
    """Gauss-Legendre in cos(theta) x uniform in phi: (theta, phi, weight) flat arrays."""
    x, w = np.polynomial.legendre.leggauss(nth)
    th = np.arccos(x)
    ph = 2.0 * np.pi * np.arange(nph) / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    W = np.repeat(w[:, None], nph, axis=1) * (2.0 * np.pi / nph)
    return T.ravel(), P.ravel(), W.ravel()


def rot_z(a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_y(b: float) -> np.ndarray:
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rotation(theta: float, phi: float, psi: float) -> np.ndarray:
    """Active rotation taking the beam frame to the sky: R = R_z(phi) R_y(theta) R_z(psi)."""
    return rot_z(phi) @ rot_y(theta) @ rot_z(psi)


def euler_of(R: np.ndarray):
    """(theta, phi, psi) with R = R_z(phi) R_y(theta) R_z(psi); theta in [0, pi]."""
    theta = float(np.arccos(np.clip(R[2, 2], -1.0, 1.0)))
    if np.sin(theta) > 1e-12:
        phi = float(np.arctan2(R[1, 2], R[0, 2]))
        psi = float(np.arctan2(R[2, 1], -R[2, 0]))
    else:  # gimbal lock: only phi +- psi is defined; put it all in phi
        phi = float(np.arctan2(R[1, 0], R[0, 0])) if R[2, 2] > 0 else float(np.arctan2(-R[1, 0], -R[0, 0]))
        psi = 0.0
    return theta, phi % (2 * np.pi), psi % (2 * np.pi)


def _xyz(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=0)


def _angles(v):
    th = np.arccos(np.clip(v[2], -1.0, 1.0))
    ph = np.arctan2(v[1], v[0]) % (2 * np.pi)
    return th, ph


def conv_quadrature(alm, blm, lmax: int, kmax: int, ptg) -> np.ndarray:
    """c = integral of s(n) b(R^{-1} n) dOmega by a grid exact for degree 2 lmax."""
    ptg = np.asarray(ptg, dtype=np.float64).reshape(-1, 3)
    th, ph, w = gl_sphere_grid(lmax + 2, 2 * lmax + 3)
    s = field_values(alm, lmax, lmax, th, ph)
    n = _xyz(th, ph)
    out = np.empty(ptg.shape[0])
    for t, (theta, phi, psi) in enumerate(ptg):
        R = rotation(theta, phi, psi)
        nb = R.T @ n
        bt, bp = _angles(nb)
        out[t] = np.sum(w * s * field_values(blm, lmax, kmax, bt, bp))
    return out


def analyse(func, lmax: int, mmax: int | None = None) -> np.ndarray:
    """a_lm = integral f(n) conj(Y_lm(n)) dOmega for a band-limited f(xyz) (exact quadrature)."""
    mmax = lmax if mmax is None else mmax
    th, ph, w = gl_sphere_grid(lmax + 2, 2 * lmax + 3)
    f = func(_xyz(th, ph))
    out = np.zeros(n_alm(lmax, mmax), dtype=np.complex128)
    for m in range(mmax + 1):
        for l in range(m, lmax + 1):
            out[alm_index(lmax, l, m)] = np.sum(w * f * np.conj(sph_harm_y(l, m, th, ph)))
    return out


def beam_moments(blm, lmax: int, kmax: int):
    """S_i = int n_i b dOmega and S_ij = int n_i n_j b dOmega (beam frame)."""
    th, ph, w = gl_sphere_grid(lmax + 3, 2 * lmax + 5)
    b = field_values(blm, lmax, kmax, th, ph)
    n = _xyz(th, ph)
    S = np.array([np.sum(w * b * n[i]) for i in range(3)])
    S2 = np.array([[np.sum(w * b * n[i] * n[j]) for j in range(3)] for i in range(3)])
    return S, S2
