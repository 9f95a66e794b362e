"""ctypes binding of libsidelobe.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only passes device
pointers, sizes and the current torch stream across the C ABI declared in
include/sidelobe.h.  It raises if the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsidelobe.so")

SC_OK, SC_EINVAL, SC_ENOMEM, SC_EHIP, SC_ESTATE = 0, -1, -2, -3, -4
SC_FP64, SC_F64MAPS_F32GATHER, SC_MIXED = 0, 1, 2

SC_PARAM_BIN_CHUNK, SC_PARAM_GATHER_WGS_PER_CU, SC_PARAM_RING_RPT, SC_PARAM_SKY_LMAX, SC_PARAM_GATHER_WAVES = 1, 2, 3, 4, 5
SC_PARAM_GATHER_MMA = 6
SC_PARAM_VALIDATE = 7
SC_PARAM_DETERMINISTIC = 8
SC_PARAM_BATCH_CHAINS = 9
SC_MMA_FP32, SC_MMA_SPLIT16 = 0, 1

EXPORTS = (
    "sc_plan_create", "sc_plan_destroy", "sc_plan_set_stream", "sc_plan_info", "sc_set_sky_beam",
    "sc_interpolate", "sc_interpolate_noalloc", "sc_plan_build_psi_cube", "sc_interpolate_psi", "sc_plan_convolve", "sc_convolve", "sc_convolve_release_cache", "sc_dipole_response", "sc_convolve_adjoint", "sc_convolve_adjoint_beam", "sc_debug_copy_stage", "sc_plan_enable_timing",
    "sc_plan_stage_times", "sc_plan_set_param", "sc_plan_get_param", "sc_batch_create", "sc_batch_run",
    "sc_batch_set_param", "sc_batch_get_param", "sc_batch_set_stream", "sc_batch_plan", "sc_batch_destroy", "sc_strerror",
    "sc_last_error",
)


class DetDesc(ctypes.Structure):
    """sc_det_desc."""
    _fields_ = [("lmax", ctypes.c_int), ("kmax", ctypes.c_int), ("blm", ctypes.c_void_p),
                ("ptg", ctypes.c_void_p), ("n", ctypes.c_int64), ("tod", ctypes.c_void_p)]

_lib = None


class ScError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load()
        msg = lib.sc_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%d): %s" % (where, lib.sc_strerror(code).decode(), code, msg))
        self.code = code


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsidelobe.so is not built; run `python -m paper_2201_03478_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.sc_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, vp]
    lib.sc_plan_destroy.argtypes = [vp]
    lib.sc_plan_set_stream.argtypes = [vp, vp]
    lib.sc_plan_info.argtypes = [vp, ctypes.POINTER(i64), i32]
    lib.sc_set_sky_beam.argtypes = [vp, vp, vp]
    lib.sc_interpolate.argtypes = [vp, vp, i64, vp]
    lib.sc_interpolate_noalloc.argtypes = [vp, vp, i64, vp]
    lib.sc_plan_convolve.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.sc_plan_build_psi_cube.argtypes = [vp, i32]
    lib.sc_interpolate_psi.argtypes = [vp, vp, i64, vp]
    f64 = ctypes.c_double
    lib.sc_dipole_response.argtypes = [vp, i32, i32, vp, i64, vp, i64, f64, f64, vp, vp]
    lib.sc_convolve.argtypes = [vp, vp, i32, i32, vp, i64, vp, i32, vp]
    lib.sc_convolve_release_cache.argtypes = []
    lib.sc_convolve_adjoint.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.sc_convolve_adjoint_beam.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.sc_debug_copy_stage.argtypes = [vp, i32, vp, i64]
    lib.sc_debug_copy_stage.restype = i64
    lib.sc_plan_enable_timing.argtypes = [vp, i32]
    lib.sc_plan_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
    lib.sc_plan_set_param.argtypes = [vp, i32, i64]
    lib.sc_plan_get_param.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.sc_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(DetDesc), i32, i32, i32, vp]
    lib.sc_batch_run.argtypes = [vp, vp, i32]
    lib.sc_batch_set_param.argtypes = [vp, i32, i32, i64]
    lib.sc_batch_get_param.argtypes = [vp, i32, i32, ctypes.POINTER(i64)]
    lib.sc_batch_set_stream.argtypes = [vp, vp]
    lib.sc_batch_plan.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.sc_batch_destroy.argtypes = [vp]
    lib.sc_strerror.argtypes = [i32]
    lib.sc_strerror.restype = ctypes.c_char_p
    lib.sc_last_error.argtypes = []
    lib.sc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code: int, where: str) -> int:
    if code < 0:
        raise ScError(code, where)
    return code
