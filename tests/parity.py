"""Parity measures of the GPU tests against the CPU oracle.

A result c_gpu is compared with the oracle's c on the same samples by
  * rel-L2   = ||c_gpu - c||_2 / ||c||_2 over the checked samples, and
  * max-rel  = max |c_gpu - c| / max |c|  (every sample, so a single bad sample
               cannot hide in the norm).
The forms' targets are stated as rel-L2 (1e-6 for the FP32 forms, 1e-12 for the
FP64 form); the element-wise bar defaults to ten times that.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _real(x):
    x = np.asarray(x)
    if np.iscomplexobj(x):  # complex coefficients: compare real and imaginary parts
        return np.ascontiguousarray(x, dtype=np.complex128).view(np.float64).ravel()
    return np.asarray(x, dtype=np.float64).ravel()


def errors(got, ref):
    got = _real(got)
    ref = _real(ref)
    assert got.shape == ref.shape
    d = got - ref
    if not np.all(np.isfinite(got)):
        return float("inf"), float("inf")
    return float(np.linalg.norm(d) / np.linalg.norm(ref)), float(np.max(np.abs(d)) / np.max(np.abs(ref)))


def assert_parity(got, ref, rel_tol: float, label: str = "", max_tol: float | None = None):
    """rel-L2 <= rel_tol and max-rel <= max_tol (default 10 rel_tol); returns both."""
    max_tol = 10.0 * rel_tol if max_tol is None else max_tol
    rel, mx = errors(got, ref)
    print("%s: rel-L2 %.3e (bar %.0e), max|d|/max|c| %.3e (bar %.0e), %d samples"
          % (label, rel, rel_tol, mx, max_tol, np.size(ref)))
    assert rel <= rel_tol, "%s: rel-L2 %.3e > %.0e" % (label, rel, rel_tol)
    assert mx <= max_tol, "%s: max|d|/max|c| %.3e > %.0e" % (label, mx, max_tol)
    return rel, mx


def coef_hash(*arrays) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.complex128).tobytes())
    return h.hexdigest()[:16]


def load_golden(workload: str):
    """Stored oracle values (tests/golden/oracle_<workload>.txt) as a list of per-detector
    dicts: det, lmax, kmax, n, coef_sha, idx [m], ptg [m, 3], c [m]."""
    path = os.path.join(GOLDEN, "oracle_%s.txt" % workload)
    dets, rows = {}, {}
    for line in open(path):
        if line.startswith("# det "):
            f = line[2:].split()
            d = int(f[1])
            dets[d] = dict(det=d, lmax=int(f[3]), kmax=int(f[5]), n=int(f[7]), coef_sha=f[9])
            rows[d] = []
        elif line.startswith("#") or not line.strip():
            continue
        else:
            f = line.split()
            rows[int(f[0])].append([float(x) for x in f[1:]])
    out = []
    for d in sorted(dets):
        r = np.array(rows[d])
        g = dets[d]
        g["idx"] = r[:, 0].astype(np.int64)
        g["ptg"] = np.ascontiguousarray(r[:, 1:4])
        g["c"] = r[:, 4]
        out.append(g)
    return out


def place_golden(torch, ptg, g):
    """Write the stored pointings into the device pointing array at their sample indices
    (they equal the scan's there, up to the last bits of its cos/sin, except the edge
    pointings); returns the index tensor."""
    it = torch.as_tensor(g["idx"], device=ptg.device)
    ptg[it] = torch.as_tensor(g["ptg"], device=ptg.device)
    return it
