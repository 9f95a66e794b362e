"""CPU-side checks of the C ABI: the library loads and exports every symbol
declared in include/sidelobe.h; argument validation that needs no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sidelobe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_03478_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        from paper_2201_03478_amd import build
        build.build()
    return N.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "sc_convolve" in names and "sc_plan_create" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_2201_03478_amd import _native as N
    assert set(names) == set(N.EXPORTS)


def test_strerror_texts(lib):
    for code in (0, -1, -2, -3, -4, -99):
        assert len(lib.sc_strerror(code)) > 0


def test_plan_create_rejects_bad_arguments_without_device(lib):
    """Validation happens before any device call, so it works without a GPU."""
    from paper_2201_03478_amd import _native as N
    p = ctypes.c_void_p()
    cases = [(-1, 0, 0, 0), (10, -1, 0, 0), (10, 11, 0, 0), (10, 2, 7, 0), (10, 2, 3, 0), (10, 2, 0, 5), (10, 2, 0, 18),
             (10, 2, 0, 3), (8193, 2, 0, 0), (20000, 2, 0, 0), (500, 128, 1, 0)]
    for lmax, kmax, prec, w in cases:
        rc = lib.sc_plan_create(ctypes.byref(p), lmax, kmax, prec, w, None)
        assert rc == N.SC_EINVAL, (lmax, kmax, prec, w)
        assert len(lib.sc_last_error()) > 0
    assert lib.sc_plan_create(None, 4, 2, 0, 0, None) == N.SC_EINVAL


def test_null_plan_calls(lib):
    from paper_2201_03478_amd import _native as N
    assert lib.sc_plan_destroy(None) == N.SC_OK
    assert lib.sc_set_sky_beam(None, None, None) == N.SC_EINVAL
    assert lib.sc_interpolate(None, None, 0, None) == N.SC_EINVAL
    assert lib.sc_plan_build_psi_cube(None, 0) == N.SC_EINVAL
    assert lib.sc_interpolate_psi(None, None, 0, None) == N.SC_EINVAL
    assert lib.sc_plan_info(None, None, 0) == N.SC_EINVAL


def test_header_constants_match_binding():
    """Every enum constant of include/sidelobe.h that the Python binding names has the
    header's value (status codes, precisions, parameters, product forms)."""
    from paper_2201_03478_amd import _native as N
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sidelobe.h")).read(), flags=re.S)
    consts = dict((k, int(v)) for k, v in re.findall(r"\b(SC_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    assert len(consts) >= 15
    named = [k for k in consts if hasattr(N, k)]
    assert "SC_PARAM_VALIDATE" in named and "SC_EINVAL" in named
    for k in named:
        assert getattr(N, k) == consts[k], k
