"""MI355X-native spin-harmonic total convolution (sidelobe convolution).

Galloway et al. (2022), "BeyondPlanck VIII", Sec. 2.1: a sky a_lm and a beam
b_lk (|k| <= kmax) give 2 kmax + 1 spin component maps by spin transforms; the
time-ordered signal at each pointing (theta, phi, psi) follows by
interpolating those maps and summing the cos k psi / sin k psi terms.

The arithmetic lives in the HIP library libsidelobe.so (C ABI in
include/sidelobe.h); ``api`` is a thin torch-facing binding, imported on first
use so that importing the package has no torch/HIP side effects.
"""
import importlib

from ._native import SC_F64MAPS_F32GATHER, SC_FP64, SC_MIXED  # noqa: F401


def __getattr__(name):
    if name in ("api", "Plan", "convolve"):
        mod = importlib.import_module(__name__ + ".api")
        return mod if name == "api" else getattr(mod, name)
    raise AttributeError(name)
