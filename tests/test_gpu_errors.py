"""Failure handling on the device side: a failed allocation returns SC_ENOMEM and
gives back what was already allocated.

The library's allocation counter (environment variable SC_FAIL_ALLOC_AFTER=k:
every allocation after the first k of the process fails) is read once per
process, so each case runs in a child process of its own.  No kernel runs in
these cases: the failures happen before any launch.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, sys
import torch
sys.path.insert(0, %(root)r)
from paper_2201_03478_amd import _native as N
torch.cuda.init()
torch.cuda.synchronize()
lib = N.load()
free0 = torch.cuda.mem_get_info()[0]
p = ctypes.c_void_p()
rc = lib.sc_plan_create(ctypes.byref(p), 512, 100, 1, 0, None)
msg = lib.sc_last_error().decode()
torch.cuda.synchronize()
free1 = torch.cuda.mem_get_info()[0]
print("RESULT", rc, p.value or 0, free0 - free1, msg, flush=True)
"""


@pytest.mark.parametrize("k", [0, 1, 2, 5])
def test_plan_create_allocation_failure(k):
    """Plan creation (lmax 512, kmax 100: ring sums 0.9 GB, spectra 1.8 GB, maps 2 GB first)
    with the (k+1)-th allocation failing: SC_ENOMEM, no plan, and device memory back where it
    was (within 64 MiB of allocator granularity, far below the 0.9 GB of the first buffer)."""
    env = dict(os.environ, SC_FAIL_ALLOC_AFTER=str(k))
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT}], env=env, capture_output=True, text=True,
                       timeout=300)
    line = [s for s in r.stdout.splitlines() if s.startswith("RESULT")]
    assert r.returncode == 0 and line, r.stdout + r.stderr
    _, rc, handle, used, msg = line[0].split(" ", 4)
    print("k=%d: rc %s, memory still held %s bytes, %s" % (k, rc, used, msg))
    assert int(rc) == -2  # SC_ENOMEM
    assert int(handle) == 0
    assert "hipMalloc" in msg
    assert abs(int(used)) <= 64 << 20
