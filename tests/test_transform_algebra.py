"""Host-side checks of the transform algebra the theta kernels rely on (CPU).

The theta stage extends each ring-sum column F_k(., m) to the full circle with
the parity F(-theta) = (-1)^{m-k} F(theta) (from d^l_mk(-theta) =
(-1)^{m-k} d^l_mk(theta)), transforms it, divides by the interpolation
kernel's transform and upsamples (the finite-resolution grid of Galloway et
al. 2022, Sec. 2.1).  The kernels transform two columns of opposite parity
with one complex FFT pair and separate them afterwards.  These tests restate
that separation with numpy FFTs on random columns and compare it with the
column-by-column computation, and check that the paired adjoint is the
transpose of the paired forward map (dot-product identity).  They pin the
identities, not the HIP code; the GPU tests compare the HIP path with the
oracle.
"""
import numpy as np
import pytest


def _setup(lmax=20, n2=44, nos=90, W=8, seed=1):
    rng = np.random.default_rng(seed)
    n = np.arange(-lmax, lmax + 1)
    q = rng.uniform(0.5, 2.0, lmax + 1)          # a real, even kernel factor
    phase = np.exp(-1j * np.pi * n / n2) * q[np.abs(n)]  # half-ring shift times 1/kernel
    dphi = rng.uniform(0.5, 2.0, lmax + 1)
    rows = nos // 2 + W
    r0 = -W // 2 + 1
    return dict(lmax=lmax, n2=n2, nos=nos, rows=rows, r0=r0, n=n, phase=phase, dphi=dphi, rng=rng)


def _single(S, Fc, m, k):
    """One column: parity extension, FFT, deconvolution, zero padding, inverse FFT, kept rows."""
    n2, nos, n = S["n2"], S["nos"], S["n"]
    nring = n2 // 2
    s = -1.0 if (m - k) & 1 else 1.0
    f = np.zeros(n2, complex)
    f[:nring] = Fc
    f[n2 - 1 - np.arange(nring)] = s * Fc
    X = np.fft.fft(f)
    Y = np.zeros(nos, complex)
    Y[n % nos] = X[n % n2] * S["phase"] * S["dphi"][abs(m)]
    O = np.fft.ifft(Y) * nos
    return O[(np.arange(S["rows"]) + S["r0"]) % nos]


def _paired(S, F1, F2, m, k, two=True):
    """Columns m and m + 1 through one forward and one inverse transform (the kernels' scheme)."""
    n2, nos, n = S["n2"], S["nos"], S["n"]
    nring = n2 // 2
    s1 = -1.0 if (m - k) & 1 else 1.0
    if not two:
        F2 = np.zeros_like(F1)
    j = np.arange(nring)
    h = np.zeros(n2, complex)
    h[j] = F1 + 1j * F2
    h[n2 - 1 - j] = s1 * (F1 - 1j * F2)
    H = np.fft.fft(h)
    d1 = S["dphi"][abs(m)]
    d2 = S["dphi"][abs(m + 1)] if two else d1
    ca, cb = 0.25 * (d1 + d2), 0.25 * s1 * (d1 - d2)
    Z = ca * S["phase"] * H[n % n2] + cb * np.conj(S["phase"]) * H[(-n) % n2]
    B = np.zeros(nos, complex)
    B[n % nos] = Z
    O = np.fft.ifft(B) * nos
    r = (np.arange(S["rows"]) + S["r0"]) % nos
    rm = (-r) % nos
    return O[r] + s1 * O[rm], -1j * (O[r] - s1 * O[rm])


def _paired_adjoint(S, G1, G2, m, k, two=True):
    n2, nos, n, rows, r0 = S["n2"], S["nos"], S["n"], S["rows"], S["r0"]
    nring = n2 // 2
    s1 = -1.0 if (m - k) & 1 else 1.0
    if not two:
        G2 = np.zeros_like(G1)
    rtop = r0 + rows - 1

    def row_of(r):
        return r - r0 if r <= rtop else (r - nos - r0 if r - nos >= r0 else -1)

    h = np.zeros(nos, complex)
    for r in range(nos):
        a, b = row_of(r), row_of((nos - r) % nos)
        a1 = G1[a] if a >= 0 else 0
        a2 = G2[a] if a >= 0 else 0
        b1 = G1[b] if b >= 0 else 0
        b2 = G2[b] if b >= 0 else 0
        h[r] = (a1 + s1 * b1) + 1j * (a2 - s1 * b2)
    Y = np.fft.fft(h)
    d1 = S["dphi"][abs(m)]
    d2 = S["dphi"][abs(m + 1)] if two else d1
    ca, cb = 0.25 * (d1 + d2), 0.25 * s1 * (d1 - d2)
    Z = np.conj(S["phase"]) * (ca * Y[n % nos] + cb * Y[(-n) % nos])
    B = np.zeros(n2, complex)
    B[n % n2] = Z
    f = np.fft.ifft(B) * n2
    j = np.arange(nring)
    return f[j] + s1 * f[n2 - 1 - j], -1j * (f[j] - s1 * f[n2 - 1 - j])


@pytest.mark.parametrize("m,k", [(-20, 0), (-3, 2), (0, 3), (5, 1), (19, 4)])
def test_paired_columns_match_single_columns(m, k):
    S = _setup()
    nring = S["n2"] // 2
    rng = S["rng"]
    F1 = rng.standard_normal(nring) + 1j * rng.standard_normal(nring)
    F2 = rng.standard_normal(nring) + 1j * rng.standard_normal(nring)
    g1, g2 = _paired(S, F1, F2, m, k)
    ref1, ref2 = _single(S, F1, m, k), _single(S, F2, m + 1, k)
    scale = max(np.abs(ref1).max(), np.abs(ref2).max())
    assert np.abs(g1 - ref1).max() <= 1e-13 * scale
    assert np.abs(g2 - ref2).max() <= 1e-13 * scale


def test_last_column_alone():
    """An odd column count leaves the last column without a partner (f2 = 0, d2 = d1)."""
    S = _setup()
    F1 = S["rng"].standard_normal(S["n2"] // 2) + 0j
    g1, _ = _paired(S, F1, None, 20, 3, two=False)
    ref = _single(S, F1, 20, 3)
    assert np.abs(g1 - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("m,k", [(-20, 0), (-1, 1), (4, 3)])
def test_paired_adjoint_is_the_transpose(m, k):
    S = _setup(seed=7)
    nring, rows, rng = S["n2"] // 2, S["rows"], S["rng"]
    F1 = rng.standard_normal(nring) + 1j * rng.standard_normal(nring)
    F2 = rng.standard_normal(nring) + 1j * rng.standard_normal(nring)
    G1 = rng.standard_normal(rows) + 1j * rng.standard_normal(rows)
    G2 = rng.standard_normal(rows) + 1j * rng.standard_normal(rows)
    g1, g2 = _paired(S, F1, F2, m, k)
    a1, a2 = _paired_adjoint(S, G1, G2, m, k)
    ip = lambda u, v: np.real(np.vdot(u, v))
    lhs = ip(g1, G1) + ip(g2, G2)
    rhs = ip(F1, a1) + ip(F2, a2)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------------------
# The psi cube: the series over k of one pixel's cos/sin components on an npsi-point
# grid, divided by the kernel transform, with two pixels packed into one complex
# inverse transform of a Hermitian spectrum; interpolating it with the kernel
# reproduces the series at any psi.

def _es(z, beta):
    q = 1.0 - z * z
    return np.where(q > 0, np.exp(beta * (np.sqrt(np.maximum(q, 0.0)) - 1.0)), 0.0)


def _kernel_transform(k, npsi, W, beta):
    """hhat(k) = int w(y / (W/2)) cos(2 pi k y / npsi) dy over grid units y (midpoint rule)."""
    y = (np.arange(200000) + 0.5) / 200000 * W - W / 2
    return np.sum(_es(y / (W / 2), beta) * np.cos(2 * np.pi * k * y / npsi)) * (W / 200000)


def _packed_cube(A, B, g, npsi):
    """Two pixels (rows of A, B) through one complex inverse transform, as the cube kernel does."""
    kmax = A.shape[1] - 1
    X = np.zeros(npsi, complex)
    for k in range(kmax + 1):
        if k == 0:
            X[0] = g[0] * (A[0, 0] + 1j * A[1, 0])
            continue
        ya = 0.5 * g[k] * (A[0, k] - 1j * B[0, k])
        yb = 0.5 * g[k] * (A[1, k] - 1j * B[1, k])
        X[k] = ya + 1j * yb
        X[npsi - k] = np.conj(ya) + 1j * np.conj(yb)
    c = np.fft.ifft(X) * npsi
    return c.real, c.imag


@pytest.mark.parametrize("kmax,npsi", [(0, 8), (3, 16), (10, 45), (20, 90)])
def test_psi_series_two_pixels_per_transform(kmax, npsi):
    rng = np.random.default_rng(kmax)
    A = rng.standard_normal((2, kmax + 1))
    B = rng.standard_normal((2, kmax + 1))
    B[:, 0] = 0.0  # the stored sin 0 psi map is zero
    g = rng.uniform(0.5, 2.0, kmax + 1)
    ca, cb = _packed_cube(A, B, g, npsi)
    psi = 2 * np.pi * np.arange(npsi) / npsi
    k = np.arange(kmax + 1)[:, None]
    for c, p in ((ca, 0), (cb, 1)):
        ref = np.sum(g[:, None] * (A[p][:, None] * np.cos(k * psi) + B[p][:, None] * np.sin(k * psi)), axis=0)
        assert np.abs(c - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("W,tol", [(8, 2e-7), (14, 1e-12)])
def test_psi_interpolation_reproduces_series(W, tol):
    """Deconvolved grid series + periodic halo + kernel weights in psi = the series, within the
    kernel's accuracy for twofold oversampling (beta = 2.3 W)."""
    kmax = 12
    npsi = 2 * (2 * kmax + 1) + 0  # 50 = 2 * 5^2
    beta = 2.30 * W
    half = W // 2
    rng = np.random.default_rng(W)
    A = rng.standard_normal((2, kmax + 1))
    B = rng.standard_normal((2, kmax + 1))
    B[:, 0] = 0.0
    g = np.array([1.0 / _kernel_transform(k, npsi, W, beta) for k in range(kmax + 1)])
    ca, _ = _packed_cube(A, B, g, npsi)
    # stored entry s holds grid point (s - W/2 + 1) mod npsi
    ext = np.array([ca[(s - half + 1) % npsi] for s in range(npsi + W - 1)])
    k = np.arange(kmax + 1)
    scale = np.sum(np.abs(A[0]) + np.abs(B[0]))
    for psi in np.concatenate([rng.uniform(0, 2 * np.pi, 40), [0.0, 2 * np.pi - 1e-12]]):
        x = psi * npsi / (2 * np.pi)
        p0 = int(np.floor(x)) - half + 1
        nodes = p0 + np.arange(W)
        w = _es((x - nodes) / half, beta)
        got = np.dot(w, ext[nodes + half - 1])
        ref = np.sum(A[0] * np.cos(k * psi) + B[0] * np.sin(k * psi))
        assert abs(got - ref) <= tol * scale, psi


# ---------------------------------------------------------------------------
# Split transforms (band limits whose transforms exceed one workgroup's LDS): a
# length n = P N transform as P length-N transforms of folded, twiddled inputs,
#   X[P k + s] = sum_j w_N^{j k} y_s[j],  y_s[j] = w_n^{j s} sum_q x[j + N q] w_P^{q s},
# for both signs of the exponent; and the single-column theta stage built from them
# against the column-by-column reference above, with its adjoint.

def _split_dft(x, P, sign):
    n = x.size
    N = n // P
    out = np.empty(n, complex)
    j = np.arange(N)
    for s in range(P):
        fold = sum(x[j + N * q] * np.exp(sign * 2j * np.pi * q * s / P) for q in range(P))
        y = fold * np.exp(sign * 2j * np.pi * j * s / n)
        out[s::P] = np.fft.fft(y) if sign < 0 else np.fft.ifft(y) * N
    return out


@pytest.mark.parametrize("n,P", [(12, 2), (30, 3), (40, 4), (90, 5), (72, 8), (17280, 2), (34560, 4)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_split_transform_identity(n, P, sign):
    x = np.random.default_rng(n + P).standard_normal(n) + 1j * np.random.default_rng(n - P).standard_normal(n)
    ref = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * n
    assert np.max(np.abs(_split_dft(x, P, sign) - ref)) <= 1e-12 * np.max(np.abs(ref))


def _single_split(S, Fc, m, k, P1, P2):
    """The single-column theta stage of the split kernels: split forward transform of the
    extended column, d p(n) on |n| <= lmax, split inverse of the zero-padded spectrum."""
    n2, nos, n, lmax = S["n2"], S["nos"], S["n"], S["lmax"]
    nring = n2 // 2
    s = -1.0 if (m - k) & 1 else 1.0
    x = np.concatenate([Fc, s * Fc[::-1]])
    X = _split_dft(x, P1, -1)
    Z = np.zeros(nos, complex)
    Z[n % nos] = X[n % n2] * S["phase"] * S["dphi"][abs(m)]
    O = _split_dft(Z, P2, 1)
    rows = np.arange(S["rows"]) + S["r0"]
    return O[rows % nos]


def _single_split_adjoint(S, Gc, m, k, P1, P2):
    n2, nos, n = S["n2"], S["nos"], S["n"]
    nring = n2 // 2
    s = -1.0 if (m - k) & 1 else 1.0
    A = np.zeros(nos, complex)
    rows = np.arange(S["rows"]) + S["r0"]
    np.add.at(A, rows % nos, Gc)
    Y = _split_dft(A, P2, -1)
    Xa = np.zeros(n2, complex)
    Xa[n % n2] = Y[n % nos] * np.conj(S["phase"]) * S["dphi"][abs(m)]
    xa = _split_dft(Xa, P1, 1)
    return xa[:nring] + s * xa[n2 - 1 - np.arange(nring)]


@pytest.mark.parametrize("m,k", [(3, 1), (-4, 2), (0, 0), (20, 5)])
def test_split_single_column_matches_reference_and_adjoint(m, k):
    S = _setup(lmax=20, n2=44, nos=88, W=8, seed=7)
    rng = S["rng"]
    Fc = rng.standard_normal(22) + 1j * rng.standard_normal(22)
    ref = _single(S, Fc, m, k)
    for P1, P2 in ((1, 1), (2, 2), (4, 4), (2, 8)):
        got = _single_split(S, Fc, m, k, P1, P2)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        # <G, T F> = <T^* G, F> with <u, v> = Re sum conj(u) v
        Gc = rng.standard_normal(S["rows"]) + 1j * rng.standard_normal(S["rows"])
        lhs = np.real(np.vdot(Gc, got))
        rhs = np.real(np.vdot(_single_split_adjoint(S, Gc, m, k, P1, P2), Fc))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
