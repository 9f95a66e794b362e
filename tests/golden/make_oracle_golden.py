"""Write oracle_<workload>.txt: direct-sum values of Eq. 2 at sampled pointings of
the full-size scan workloads, for the GPU parity tests.

Every value comes from ``oracle.convolve`` (the plain long-double sum of Eq. 2 of
Galloway et al. 2022, Sec. 2.1) on the seeded sky and beam of the workload and
on the exact pointings stored in the file.  The pointings are the synthetic
scan's at seeded random sample indices (plus the first and last sample); a few
of them are replaced by edge pointings (the poles, phi and psi next to 2 pi,
theta on the scan's turning circles), which the GPU test writes into its
pointing array at the same indices before it runs.

Nothing here touches the HIP library.  Rerun with

    python tests/golden/make_oracle_golden.py [workload ...]

(about 20 minutes on 8 cores for all of them).
"""
import hashlib
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from workloads.generators import _scan_block, truncate_alm  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# Edge pointings written over the scan at the first sampled indices (theta, phi, psi).
EDGES = [
    (0.0, 0.3, 1.0), (math.pi, 2.0, 0.5), (1e-9, 2 * math.pi - 1e-13, 3.0), (math.pi - 1e-9, 0.0, 2 * math.pi - 1e-13),
    (math.radians(5.0), 2 * math.pi - 1e-15, 0.0), (math.radians(175.0), 1e-15, 6.283185307179586),
    (0.5 * math.pi, 0.0, 0.0), (1.0, math.pi, math.pi),
]

# name: (config number, lmax, kmax, n, samples, edges, [detector index or None])
WORKLOADS = {
    "sidelobe-lmax512-kmax100-scan1e7": (2, 512, 100, 10_000_000, 2000, True, None),
    "precision-lmax1024-kmax16-scan1e8": (3, 1024, 16, 100_000_000, 200, True, None),
    "adjoint-lmax512-kmax32-scan1e8": (5, 512, 32, 100_000_000, 200, True, None),
    "batched-12det-scan4e7": (4, None, None, None, 50, False, "all"),
}


def coef_hash(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.complex128).tobytes())
    return h.hexdigest()[:16]


def sample_pointings(n, m, seed, t0, psi0, edges):
    idx = np.sort(np.random.default_rng(seed).choice(n, m, replace=False))
    idx[0], idx[-1] = 0, n - 1
    idx = np.unique(idx)
    ptg = _scan_block(np, idx.astype(np.float64), t0, psi0)
    if edges:
        for j, e in enumerate(EDGES):
            ptg[1 + j] = e
    return idx, ptg


def write(path, header, det, idx, ptg, val):
    with open(path, "a") as f:
        for line in header:
            f.write("# %s\n" % line)
        for i in range(idx.size):
            f.write("%d %d %.17e %.17e %.17e %.17e\n" % (det, idx[i], ptg[i, 0], ptg[i, 1], ptg[i, 2], val[i]))


def make(name, nthreads=0):
    cfg, L, K, n, m, edges, dets = WORKLOADS[name]
    path = os.path.join(HERE, "oracle_%s.txt" % name)
    if os.path.exists(path):
        os.remove(path)
    t = time.time()
    with open(path, "w") as f:
        f.write("# Direct sum of Eq. 2 (Galloway et al. 2022, Sec. 2.1) from oracle.convolve, long double.\n")
        f.write("# workload %s; written by tests/golden/make_oracle_golden.py\n" % name)
        f.write("# columns: detector sample_index theta phi psi c\n")
    if dets is None:
        a = W.sky_alm(L, W.config_seed(cfg, 1))
        b = W.beam_alm(L, K, W.config_seed(cfg, 2), kind="sidelobe")
        idx, ptg = sample_pointings(n, m, W.config_seed(cfg, 6), 0.0, 0.0, edges)
        val = oracle.convolve(a, b, L, K, ptg, nthreads=nthreads)
        write(path, ["det 0 lmax %d kmax %d n %d coef_sha %s" % (L, K, n, coef_hash(a, b))], 0, idx, ptg, val)
    else:
        sky = W.sky_alm(1024, W.config_seed(cfg, 1))
        for d, (L, K, n) in enumerate(W.DETECTORS):
            a = truncate_alm(sky, 1024, L)
            b = W.beam_alm(L, K, W.config_seed(cfg, 10 + d))
            idx, ptg = sample_pointings(n, m, W.config_seed(cfg, 100 + d), 1000.0 * d, d * math.pi / 12, False)
            val = oracle.convolve(a, b, L, K, ptg, nthreads=nthreads)
            write(path, ["det %d lmax %d kmax %d n %d coef_sha %s" % (d, L, K, n, coef_hash(a, b))], d, idx, ptg, val)
            print("  detector %d done (%.0f s)" % (d, time.time() - t), flush=True)
    print("wrote %s (%.0f s)" % (path, time.time() - t), flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(WORKLOADS):
        make(name)
