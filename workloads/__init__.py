"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the convolution method: only random
coefficients with the stated spectra and synthetic pointings.  Both the CPU
oracle's callers and the GPU path's callers draw their inputs from here.
"""
from .generators import (  # noqa: F401
    CONFIGS,
    DETECTORS,
    beam_alm,
    config_seed,
    n_alm,
    residual,
    scan_pointings,
    sky_alm,
    uniform_pointings,
)
