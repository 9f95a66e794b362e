"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (CPU only).

* The oracle (test infrastructure) with the driver oracle/sanitize_check.c, which
  runs every oracle entry point on small seeded inputs (lmax 0, kmax = lmax, the
  poles, phi = 2 pi, negative psi) and its argument errors.
* The library's host code (sc_api.cpp, sc_noalloc.cpp compiled with the sanitizers
  on the host side only, linked with the normally built kernels) with the driver
  tests/sanitize/abi_check.c, which exercises the argument checks of every entry
  point that can be refused without a device.
Any out-of-bounds access, use after free, leak, signed overflow or invalid shift
ends the driver with an error.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_03478_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", *SAN, "-o", exe,
          os.path.join(ROOT, "oracle", "sc_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_check.c"), "-lm"])
    r = _run([exe], timeout=600, env=dict(os.environ, OMP_NUM_THREADS="2"))
    assert "ran clean" in r.stdout


def test_abi_host_code_under_sanitizers(tmp_path):
    from paper_2201_03478_amd import build
    hipcc, clang = build.HIPCC, "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not available")
    objs = [os.path.join(build.BUILD, os.path.splitext(s)[0] + ".o") for s in build.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    host = []
    for src in ("sc_api.cpp", "sc_noalloc.cpp"):
        o = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        # sanitizers on the host side only (each flag behind -Xarch_host)
        _run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer", "-c", os.path.join(CSRC, src), "-o", o])
        host.append(o)
    lib = str(tmp_path / "libsidelobe_san.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-o", lib, *host, *objs])
    exe = str(tmp_path / "abi_check")
    _run([clang, "-std=c99", "-O1", "-g", *SAN, "-o", exe, os.path.join(ROOT, "tests", "sanitize", "abi_check.c"),
          lib, "-Wl,-rpath," + str(tmp_path)])
    r = _run([exe], timeout=600, cwd=str(tmp_path))
    assert "ran clean" in r.stdout
