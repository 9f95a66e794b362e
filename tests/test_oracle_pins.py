"""Pins for the CPU oracle: each test ties it to something other than itself.

Galloway et al. (2022), Sec. 2.1: the convolution integral (Eq. 1), its harmonic
form (Eq. 2), the symmetries (Eqs. 5-6), the k = 0 spin-0 special case and the
+-k pairing (Eq. 8); Sec. 3.3: the dipole/quadrupole beam-moment shortcut
(Eqs. 14-19).  Each pin is chosen so that a plausible slip in the oracle (a
dropped term, a sign, a swapped index or a missing conjugate) breaks one.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _random_coefs(lmax, mmax, seed):
    rng = _rng(seed)
    n = W.n_alm(lmax, mmax)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    # zero the imaginary part of the m = 0 entries (real fields)
    a[:lmax + 1] = a[:lmax + 1].real
    return a


# ---------------------------------------------------------------- Wigner d ---

def test_P1_wigner_d_matches_explicit_sum_small_l(oracle_lib):
    """d from the oracle's recursion = Wigner's explicit sum (mpmath), l <= 20."""
    from oracle.brute import wigner_d_explicit
    L, K = 20, 6
    for theta in (0.0, 1e-3, 0.83, math.pi / 2, 2.6, math.pi):
        d = oracle_lib.wigner_d(L, K, theta)
        for l in range(0, L + 1, 3):
            for m in range(-l, l + 1):
                for k in range(-min(l, K), min(l, K) + 1):
                    ref = float(wigner_d_explicit(l, m, k, theta, dps=50))
                    assert abs(d[k + K, m + L, l] - ref) < 1e-14, (l, m, k, theta)


def test_P1b_wigner_d_golden_moderate_l(oracle_lib):
    """Stored 120-digit explicit-sum values at l = 25, 50, 100 (tests/golden)."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "wigner_d_mpmath.txt")) if not ln.startswith("#")]
    cache = {}
    worst = 0.0
    for l, m, k, th, v in rows:
        l, m, k, th, v = int(l), int(m), int(k), float(th), float(v)
        key = (th,)
        if key not in cache:
            cache[key] = oracle_lib.wigner_d(100, 16, th)
        d = cache[key][k + 16, m + 100, l]
        worst = max(worst, abs(d - v))
    assert worst < 1e-14, worst


def test_P2_unitarity_to_l1024(oracle_lib):
    """sum_m d^l_mk(theta)^2 = 1 for every l <= 1024 (orthogonality of D)."""
    L, K = 1024, 2
    for theta in (0.0031, 0.9, 2.2, math.pi - 0.0031):
        d = oracle_lib.wigner_d(L, K, theta)
        for k in range(-K, K + 1):
            s = np.sum(d[k + K] ** 2, axis=0)  # over m
            ls = np.arange(L + 1)
            ok = ls >= abs(k)
            assert np.max(np.abs(s[ok] - 1.0)) < 1e-12, (theta, k)


@pytest.mark.parametrize("theta", [0.5 * math.pi / 8640, 1.1, math.pi - 2.5 * math.pi / 8640])
def test_P2_unitarity_at_l8192(oracle_lib, theta):
    """sum_m d^L_mk(theta)^2 = 1 at L = 8192 (the largest band limit), on the rings next to
    the poles where the start values are below 1e-30000, read through the ring sums of a sky
    and a beam that are 1 at l = L only: F_k(theta, m) = a_Lm d^L_mk(theta) with |a_Lm| = 1."""
    L, K = 8192, 2
    a = np.zeros(oracle_lib.n_alm(L), complex)
    a[[oracle_lib.alm_index(L, L, m) for m in range(L + 1)]] = 1.0
    for k0 in (0, 2):
        b = np.zeros(oracle_lib.n_alm(L, K), complex)
        b[oracle_lib.alm_index(L, L, k0)] = 1.0
        F = oracle_lib.ring_sums(a, b, L, K, [theta])[k0, 0]  # [m + L]
        assert np.all(np.isfinite(F))
        assert abs(np.sum(np.abs(F) ** 2) - 1.0) < 1e-12, (theta, k0)


def test_P2b_gauss_legendre_orthogonality(oracle_lib):
    """sum_j w_j d^l_mk(theta_j) d^l'_mk(theta_j) = 2/(2l+1) delta_ll' (exact quadrature)."""
    L, K = 40, 5
    x, w = np.polynomial.legendre.leggauss(L + 1)
    tabs = np.stack([oracle_lib.wigner_d(L, K, math.acos(xi)) for xi in x])  # [j, k, m, l]
    for m, k in ((0, 0), (3, 2), (-7, 5), (12, -4), (40, 1)):
        G = np.einsum("j,jl,jn->ln", w, tabs[:, k + K, m + L, :], tabs[:, k + K, m + L, :])
        l0 = max(abs(m), abs(k))
        ls = np.arange(L + 1)
        ref = np.diag(np.where(ls >= l0, 2.0 / (2 * ls + 1), 0.0))
        assert np.max(np.abs(G - ref)) < 1e-13, (m, k)


def test_P3_symmetries(oracle_lib):
    """d_mk = (-1)^(m-k) d_km = d_{-k,-m};  d_mk(pi - t) = (-1)^(l+m) d_{m,-k}(t)."""
    L, K = 30, 30
    t = 0.77
    d = oracle_lib.wigner_d(L, K, t)
    dr = oracle_lib.wigner_d(L, K, math.pi - t)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for k in range(-l, l + 1):
                v = d[k + K, m + L, l]
                assert abs(v - (-1) ** (m - k) * d[m + K, k + L, l]) < 1e-14
                assert abs(v - d[-m + K, -k + L, l]) < 1e-14
                assert abs(dr[k + K, m + L, l] - (-1) ** (l + m) * d[-k + K, m + L, l]) < 1e-14


def test_P4_special_angles(oracle_lib):
    """d(0) = delta_mk and d(pi) = (-1)^(l-k) delta_{m,-k}."""
    L, K = 50, 8
    d0 = oracle_lib.wigner_d(L, K, 0.0)
    dp = oracle_lib.wigner_d(L, K, math.pi)
    for l in range(L + 1):
        for k in range(-min(l, K), min(l, K) + 1):
            for m in range(-l, l + 1):
                assert d0[k + K, m + L, l] == pytest.approx(1.0 if m == k else 0.0, abs=1e-15)
                ref = (-1.0) ** (l - k) if m == -k else 0.0
                # float(pi) misses pi by 1.2e-16, so cos(theta/2) is 6e-17, not 0:
                # entries that vanish at pi exactly are O(l * 6e-17) here
                assert dp[k + K, m + L, l] == pytest.approx(ref, abs=(l + 1) * 1e-16)


# ------------------------------------------------------------ convolution ---

def test_definition_pixel_quadrature_tiny(oracle_lib):
    """Eq. 2 (oracle) = Eq. 1 evaluated in pixel space by exact quadrature, incl. poles."""
    from oracle.brute import conv_quadrature
    L, K = 6, 4
    a = _random_coefs(L, L, 11)
    b = _random_coefs(L, K, 12)
    p = W.uniform_pointings(12, 13)
    p[0] = [0.0, 0.4, 2.0]
    p[1] = [math.pi, 5.9, 0.1]
    p[2] = [1e-7, 1.0, 3.0]
    re, im = oracle_lib.convolve(a, b, L, K, p, return_imag=True)
    q = conv_quadrature(a, b, L, K, p)
    assert np.max(np.abs(re - q)) < 1e-13 * np.max(np.abs(q))
    assert np.max(np.abs(im)) < 1e-15 * np.max(np.abs(re))


def test_definition_pixel_quadrature_fp64_workload(oracle_lib):
    """The same check at the lmax = 64, kmax = 4 Gaussian-beam workload."""
    from oracle.brute import conv_quadrature
    L, K = 64, 4
    a = W.sky_alm(L, W.config_seed(1, 1))
    b = W.beam_alm(L, K, W.config_seed(1, 2), kind="gauss")
    p = W.uniform_pointings(4, 77)
    re = oracle_lib.convolve(a, b, L, K, p)
    q = conv_quadrature(a, b, L, K, p)
    assert np.max(np.abs(re - q)) < 1e-13 * np.max(np.abs(q))


def test_P5_axisymmetric_beam_is_smoothed_map(oracle_lib):
    """k = 0 only: c = sum a_lm b_l0 sqrt(4 pi/(2l+1)) Y_lm(theta, phi), independent of psi."""
    L = 64
    a = W.sky_alm(L, 5)
    b = np.zeros(W.n_alm(L, 0), dtype=np.complex128)
    b[:] = W.beam_alm(L, 0, 6, kind="gauss")
    p = W.uniform_pointings(20, 7)
    c = oracle_lib.convolve(a, b, L, 0, p)
    ref = np.zeros(len(p))
    for m in range(L + 1):
        for l in range(m, L + 1):
            y = sph_harm_y(l, m, p[:, 0], p[:, 1])
            t = a[oracle_lib.alm_index(L, l, m)] * b[l].real * math.sqrt(4 * math.pi / (2 * l + 1)) * y
            ref += t.real if m == 0 else 2.0 * t.real
    assert np.max(np.abs(c - ref)) < 1e-13 * np.max(np.abs(ref))
    p2 = p.copy()
    p2[:, 2] = (p2[:, 2] + 1.234) % (2 * math.pi)
    assert np.max(np.abs(oracle_lib.convolve(a, b, L, 0, p2) - c)) < 1e-14


def test_P6_monopole_sky_is_constant(oracle_lib):
    L, K = 20, 10
    a = np.zeros(W.n_alm(L), dtype=np.complex128)
    a[0] = 0.7
    b = _random_coefs(L, K, 3)
    c = oracle_lib.convolve(a, b, L, K, W.uniform_pointings(16, 4))
    assert np.max(np.abs(c - 0.7 * b[0].real)) < 1e-15


def test_P7_dipole_quadrupole_beam_moments(oracle_lib):
    """Sky = T0[beta.n + q (beta.n)^2]: c(R) = T0[(R^T beta).S + q (R^T beta)^T S2 (R^T beta)] (Sec. 3.3)."""
    from oracle.brute import analyse, beam_moments, rotation
    L, K = 2, 2
    beta = np.array([0.3, -0.5, 0.8])
    T0, q = 1.7, 1.25
    a = analyse(lambda n: T0 * (beta @ n + q * (beta @ n) ** 2), L)
    b = _random_coefs(L, K, 21)
    S, S2 = beam_moments(b, L, K)
    p = W.uniform_pointings(10, 22)
    p[0] = [0.0, 1.0, 0.5]
    c = oracle_lib.convolve(a, b, L, K, p)
    for t, (th, ph, ps) in enumerate(p):
        u = rotation(th, ph, ps).T @ beta
        ref = T0 * (u @ S + q * u @ S2 @ u)
        assert abs(c[t] - ref) < 1e-13, t


def test_P8_rotation_invariance(oracle_lib):
    """Rotating the sky by R0 and the pointing by R0 leaves c unchanged."""
    from oracle.brute import analyse, euler_of, field_values, rotation
    L, K = 8, 5
    a = _random_coefs(L, L, 31)
    b = _random_coefs(L, K, 32)
    R0 = rotation(0.9, 2.1, -0.4)

    def rotated_sky(n):  # s'(n) = s(R0^T n)
        v = R0.T @ n
        th = np.arccos(np.clip(v[2], -1, 1))
        ph = np.arctan2(v[1], v[0]) % (2 * np.pi)
        return field_values(a, L, L, th, ph)

    a2 = analyse(rotated_sky, L)
    p = W.uniform_pointings(8, 33)
    p2 = np.array([euler_of(R0 @ rotation(*row)) for row in p])
    c1 = oracle_lib.convolve(a, b, L, K, p)
    c2 = oracle_lib.convolve(a2, b, L, K, p2)
    assert np.max(np.abs(c1 - c2)) < 1e-13 * np.max(np.abs(c1))


def test_P9_poles(oracle_lib):
    """theta = 0: c depends on phi + psi only; theta = pi: on phi - psi only."""
    L, K = 16, 7
    a = _random_coefs(L, L, 41)
    b = _random_coefs(L, K, 42)
    p = np.array([[0.0, 0.3, 1.2], [0.0, 1.5, 0.0], [math.pi, 0.3, 1.2], [math.pi, 0.0, 0.9]])  # phi - psi = -0.9 in both
    c = oracle_lib.convolve(a, b, L, K, p)
    assert abs(c[0] - c[1]) < 1e-13 * abs(c[0])
    assert abs(c[2] - c[3]) < 1e-13 * abs(c[2])


def test_P10_psi_average_is_k0_term(oracle_lib):
    """Mean over 2 kmax + 1 uniform psi removes every k != 0 term (Eq. 8)."""
    L, K = 12, 5
    a = _random_coefs(L, L, 51)
    b = _random_coefs(L, K, 52)
    b0 = np.zeros(W.n_alm(L, 0), dtype=np.complex128)
    b0[:] = b[:L + 1]
    th, ph = 1.1, 4.0
    psis = 2 * math.pi * np.arange(2 * K + 1) / (2 * K + 1) + 0.3
    p = np.stack([np.full_like(psis, th), np.full_like(psis, ph), psis], axis=1)
    mean = oracle_lib.convolve(a, b, L, K, p).mean()
    ref = oracle_lib.convolve(a, b0, L, 0, p[:1])[0]
    assert abs(mean - ref) < 1e-13 * abs(ref)


def test_P11_so3_parseval(oracle_lib):
    """int c^2 dR = sum_l 8 pi^2/(2l+1) sum_{m,k} |a_lm|^2 |b_lk|^2 over all m, k (exact quadrature)."""
    L, K = 5, 3
    a = _random_coefs(L, L, 61)
    b = _random_coefs(L, K, 62)
    x, w = np.polynomial.legendre.leggauss(L + 1)
    nph, nps = 2 * L + 1, 2 * K + 1
    th = np.arccos(x)
    P = np.array([[t, 2 * math.pi * i / nph, 2 * math.pi * j / nps]
                  for t in th for i in range(nph) for j in range(nps)])
    wt = np.repeat(w, nph * nps) * (2 * math.pi / nph) * (2 * math.pi / nps)
    c = oracle_lib.convolve(a, b, L, K, P)
    lhs = np.sum(wt * c * c)

    def full_power(coefs, mmax, l):
        s = abs(coefs[l].real) ** 2  # m = 0 (imaginary part ignored)
        for m in range(1, min(l, mmax) + 1):
            s += 2 * abs(coefs[m * (2 * L + 1 - m) // 2 + l]) ** 2  # +m and -m
        return s

    rhs = sum(8 * math.pi ** 2 / (2 * l + 1) * full_power(a, L, l) * full_power(b, K, l) for l in range(L + 1))
    assert abs(lhs - rhs) < 1e-12 * rhs


# --------------------------------------------------- stage quantities -------

def test_component_maps_pair_into_convolution(oracle_lib):
    """c = T_0 + sum_k 2[cos k psi Re T_k - sin k psi Im T_k] (Eq. 8), T from the stage routine."""
    L, K = 20, 6
    a = _random_coefs(L, L, 71)
    b = _random_coefs(L, K, 72)
    p = W.uniform_pointings(10, 73)
    T = oracle_lib.component_maps(a, b, L, K, p[:, 0], p[:, 1])
    ks = np.arange(1, K + 1)
    c2 = T[:, 0].real + np.sum(2 * (np.cos(np.outer(p[:, 2], ks)) * T[:, 1:].real
                                    - np.sin(np.outer(p[:, 2], ks)) * T[:, 1:].imag), axis=1)
    c = oracle_lib.convolve(a, b, L, K, p)
    assert np.max(np.abs(c - c2)) < 1e-13 * np.max(np.abs(c))
    assert np.max(np.abs(T[:, 0].imag)) < 1e-14


def test_ring_sums_synthesise_component_maps(oracle_lib):
    """T_k(theta, phi) = sum_m F_k(theta, m) e^{i m phi}."""
    L, K = 15, 4
    a = _random_coefs(L, L, 81)
    b = _random_coefs(L, K, 82)
    th = np.array([0.2, 1.3, 2.9])
    ph = np.array([0.5, 3.3, 6.0])
    F = oracle_lib.ring_sums(a, b, L, K, th)
    T = oracle_lib.component_maps(a, b, L, K, th, ph)
    m = np.arange(-L, L + 1)
    for j in range(3):
        Tj = F[:, j, :] @ np.exp(1j * m * ph[j])
        assert np.max(np.abs(Tj - T[j])) < 1e-13


# ------------------------------------------------------------- adjoint -----

def test_adjoint_dot_product_and_finite_difference(oracle_lib):
    """<y, A a> = Re sum conj(A^T y) a (Z13 inner product) and FD on random entries."""
    L, K = 10, 4
    a = _random_coefs(L, L, 91)
    b = _random_coefs(L, K, 92)
    p = W.uniform_pointings(40, 93)
    y = _rng(94).standard_normal(40)
    g = oracle_lib.adjoint(b, L, K, p, y)
    lhs = float(y @ oracle_lib.convolve(a, b, L, K, p))
    rhs = float(np.real(np.sum(np.conj(g) * a)))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert np.all(g[:L + 1].imag == 0)
    # A is linear: a central difference is exact up to rounding
    rng = _rng(95)
    for idx in rng.choice(W.n_alm(L), 6, replace=False):
        for unit, part in ((1.0, "re"), (1j, "im")):
            if part == "im" and idx <= L:
                continue
            e = np.zeros_like(a)
            e[idx] = unit
            h = 1e-3
            fd = (y @ oracle_lib.convolve(a + h * e, b, L, K, p) - y @ oracle_lib.convolve(a - h * e, b, L, K, p)) / (2 * h)
            ref = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - ref) < 1e-9 * max(1.0, abs(ref)), (idx, part)


def test_P12_beam_gradient_dot_identity_and_difference(oracle_lib):
    """The beam-gradient oracle is the transpose of the forward sum in b: sum_t y_t c_t(a, b) =
    Re sum conj(h_lk) b_lk (c is linear in b), and a finite difference in one b_lk agrees."""
    L, K, n = 10, 3, 30
    a = W.sky_alm(L, 41)
    b = W.beam_alm(L, K, 42)
    b[:L + 1] = b[:L + 1].real  # the k = 0 column is real
    p = W.uniform_pointings(n, 43)
    y = _rng(44).standard_normal(n)
    h = oracle_lib.beam_adjoint(a, L, K, p, y)
    c = oracle_lib.convolve(a, b, L, K, p)
    assert abs(float(y @ c) - float(np.real(np.vdot(h, b)))) < 1e-12 * abs(float(y @ c))
    for (l, k) in ((4, 2), (7, 0)):
        i = k * (2 * L + 1 - k) // 2 + l
        for comp, unit in ((0, 1.0), (1, 1j)):
            if k == 0 and comp == 1:
                continue
            e = np.zeros_like(b)
            e[i] = unit
            dlin = float(y @ (oracle_lib.convolve(a, b + e, L, K, p) - c))  # exact: c is linear in b
            ref = h[i].real if comp == 0 else h[i].imag
            assert abs(dlin - ref) < 1e-12 * max(1.0, abs(ref)), (l, k, comp)


def test_P13_terms_below_2e600_are_negligible(oracle_lib):
    """Reading of the extended-exponent recursion: a column's contributions are counted once
    its values reach 2^-600, so the terms dropped are each below 2^-600 |a_lm b_lk|.  At
    lmax 1300 on a ring at 22.6 degrees (where the columns m ~ 430-460 start far below that)
    dropping every term with |d^l_mk| < 2^-600 from the direct sum of Eq. 2 changes c by
    less than 1e-14 relative; the sum itself is checked against the oracle's convolution."""
    L, K = 1300, 2
    theta, phi, psi = math.radians(22.6), 0.7, 1.9
    a = W.sky_alm(L, 6800)
    b = W.beam_alm(L, K, 6801)
    d = oracle_lib.wigner_d(L, K, theta)  # [k + K, m + L, l]
    A = np.zeros((2 * L + 1, L + 1), complex)  # a_lm for -l <= m <= l (Eq. 6 for m < 0)
    for m in range(L + 1):
        i0 = m * (2 * L + 1 - m) // 2
        v = a[i0 + np.arange(m, L + 1)]  # a_lm, l = m .. L (m-major layout: index m(2L+1-m)/2 + l)
        col = np.zeros(L + 1, complex)
        col[m:] = v.real if m == 0 else v
        A[L + m] = col
        if m:
            A[L - m] = (-1) ** m * np.conj(col)
    B = np.zeros((2 * K + 1, L + 1), complex)
    for k in range(K + 1):
        i0 = k * (2 * L + 1 - k) // 2
        col = np.zeros(L + 1, complex)
        col[k:] = b[i0 + np.arange(k, L + 1)]
        if k == 0:
            col = col.real.astype(complex)
        B[K + k] = col
        if k:
            B[K - k] = (-1) ** k * np.conj(col)
    ph = np.exp(1j * (np.arange(-L, L + 1)[None, :] * phi + np.arange(-K, K + 1)[:, None] * psi))
    terms = A[None, :, :] * np.conj(B)[:, None, :] * d  # [k, m, l]
    full = np.sum(ph * terms.sum(axis=2)).real
    ref = oracle_lib.convolve(a, b, L, K, np.array([[theta, phi, psi]]))[0]
    assert abs(full - ref) <= 1e-12 * abs(ref)
    small = (np.abs(d) < 2.0 ** -600) & (np.abs(A)[None, :, :] > 0)
    assert np.count_nonzero(small & (d != 0)) > 1000  # many such terms are present
    dropped = np.sum(ph * np.where(small, 0.0, terms).sum(axis=2)).real
    print("c %.15e, change from dropping |d| < 2^-600: %.3e relative" % (full, abs(dropped - full) / abs(full)))
    assert abs(dropped - full) <= 1e-14 * abs(full)
