"""CPU oracle for the spin-harmonic total convolution (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product library never does, and it
shares no code with it.

``sc_oracle.c`` evaluates the total-convolution sum of Galloway et al. (2022),
Sec. 2.1, Eq. 2, directly, in long double, for every sample; ``brute.py`` holds
the arbitrary-precision and pixel-quadrature checks that pin it.

All coefficient arrays are complex128 in the m-major triangular layout
``index(l, m) = m (2 lmax + 1 - m) / 2 + l``; the beam uses the same lmax and
stores only ``k <= kmax``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB = os.path.join(_HERE, "libsc_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.sco_wigner_d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        lib.sco_convolve.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_long,
                                     dp, dp, ctypes.c_int]
        lib.sco_ring_sums.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_long,
                                      dp, ctypes.c_int]
        lib.sco_component_maps.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                           ctypes.c_long, dp, ctypes.c_int]
        lib.sco_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_long,
                                    dp, ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_f64(a) -> np.ndarray:
    a = np.asarray(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a, dtype=np.complex128).view(np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def n_alm(lmax: int, mmax: int | None = None) -> int:
    """Number of stored coefficients for 0 <= m <= min(l, mmax), l <= lmax."""
    mmax = lmax if mmax is None else mmax
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def alm_index(lmax: int, l: int, m: int) -> int:
    return m * (2 * lmax + 1 - m) // 2 + l


def wigner_d(lmax: int, kmax: int, theta: float) -> np.ndarray:
    """d^l_{mk}(theta) as an array indexed [k + kmax, m + lmax, l]."""
    out = np.zeros((2 * kmax + 1, 2 * lmax + 1, lmax + 1), dtype=np.float64)
    rc = _load().sco_wigner_d(lmax, kmax, float(theta), _ptr(out))
    if rc != 0:
        raise ValueError("sco_wigner_d failed: %d" % rc)
    return out


def convolve(alm, blm, lmax: int, kmax: int, ptg, nthreads: int = 0, return_imag: bool = False):
    """Direct sum of Eq. 2 at each pointing (theta, phi, psi); float64 result."""
    a = _as_f64(alm)
    b = _as_f64(blm)
    p = np.ascontiguousarray(ptg, dtype=np.float64).reshape(-1, 3)
    if a.size != 2 * n_alm(lmax) or b.size != 2 * n_alm(lmax, kmax):
        raise ValueError("coefficient array sizes do not match lmax/kmax")
    n = p.shape[0]
    re = np.zeros(n)
    im = np.zeros(n)
    rc = _load().sco_convolve(lmax, kmax, _ptr(a), _ptr(b), _ptr(p), n, _ptr(re), _ptr(im), nthreads)
    if rc != 0:
        raise ValueError("sco_convolve failed: %d" % rc)
    return (re, im) if return_imag else re


def ring_sums(alm, blm, lmax: int, kmax: int, theta, nthreads: int = 0) -> np.ndarray:
    """F_k(theta_j, m) = sum_l a_lm conj(b_lk) d^l_mk(theta_j); complex [k, j, m + lmax]."""
    a = _as_f64(alm)
    b = _as_f64(blm)
    th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    out = np.zeros((kmax + 1, th.size, 2 * lmax + 1, 2))
    rc = _load().sco_ring_sums(lmax, kmax, _ptr(a), _ptr(b), _ptr(th), th.size, _ptr(out), nthreads)
    if rc != 0:
        raise ValueError("sco_ring_sums failed: %d" % rc)
    return out[..., 0] + 1j * out[..., 1]


def component_maps(alm, blm, lmax: int, kmax: int, theta, phi, nthreads: int = 0) -> np.ndarray:
    """T_k(theta, phi) = sum_{l,m} a_lm conj(b_lk) d^l_mk(theta) e^{i m phi}; complex [t, k]."""
    a = _as_f64(alm)
    b = _as_f64(blm)
    th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    ph = np.ascontiguousarray(phi, dtype=np.float64).ravel()
    out = np.zeros((th.size, kmax + 1, 2))
    rc = _load().sco_component_maps(lmax, kmax, _ptr(a), _ptr(b), _ptr(th), _ptr(ph), th.size,
                                    _ptr(out), nthreads)
    if rc != 0:
        raise ValueError("sco_component_maps failed: %d" % rc)
    return out[..., 0] + 1j * out[..., 1]


def adjoint(blm, lmax: int, kmax: int, ptg, y, nthreads: int = 0) -> np.ndarray:
    """g_lm = dL/dRe a_lm + i dL/dIm a_lm for L = sum_t y_t c_t; complex128 alm layout."""
    b = _as_f64(blm)
    p = np.ascontiguousarray(ptg, dtype=np.float64).reshape(-1, 3)
    yy = np.ascontiguousarray(y, dtype=np.float64).ravel()
    if yy.size != p.shape[0]:
        raise ValueError("y and ptg lengths differ")
    g = np.zeros(2 * n_alm(lmax))
    rc = _load().sco_adjoint(lmax, kmax, _ptr(b), _ptr(p), _ptr(yy), p.shape[0], _ptr(g), nthreads)
    if rc != 0:
        raise ValueError("sco_adjoint failed: %d" % rc)
    return g.view(np.complex128)


def beam_adjoint(alm, lmax: int, kmax: int, ptg, y) -> np.ndarray:
    """h_lk = dL/dRe b_lk + i dL/dIm b_lk for L = sum_t y_t c_t (k >= 0; h_l0 real).

    Eq. 2 with both signs of k, c = sum_{l, |k| <= kmax} conj(b_lk) X_lk with
    X_lk(t) = sum_{|m| <= l} a_lm e^{i m phi_t} d^l_mk(theta_t) e^{i k psi_t}; the
    real-field relations (Eq. 6) pair k and -k, so c = sum_l [b_l0 X_l0 +
    2 sum_{k >= 1} Re(conj(b_lk) X_lk)] and h_lk = 2 sum_t y_t X_lk (k >= 1),
    h_l0 = sum_t y_t Re X_l0.  Plain loops over samples (small cases only).
    """
    a = np.asarray(alm, dtype=np.complex128)
    p = np.ascontiguousarray(ptg, dtype=np.float64).reshape(-1, 3)
    yy = np.ascontiguousarray(y, dtype=np.float64).ravel()
    # all orders m of the real sky: a_{l,-m} = (-1)^m conj(a_lm)
    A = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            v = a[alm_index(lmax, l, m)]
            if m == 0:
                v = complex(v.real, 0.0)
            A[l, m + lmax] = v
            A[l, lmax - m] = (-1) ** m * np.conj(v)
    ms = np.arange(-lmax, lmax + 1)
    h = np.zeros(n_alm(lmax, kmax), dtype=np.complex128)
    for t in range(p.shape[0]):
        th, ph, ps = p[t]
        d = wigner_d(lmax, kmax, th)  # [k + kmax, m + lmax, l]
        em = np.exp(1j * ms * ph)
        for k in range(kmax + 1):
            X = np.einsum("lm,m,ml->l", A, em, d[k + kmax]) * np.exp(1j * k * ps)
            for l in range(k, lmax + 1):
                h[k * (2 * lmax + 1 - k) // 2 + l] += yy[t] * (
                    2.0 * X[l] if k > 0 else X[l].real)
    return h
