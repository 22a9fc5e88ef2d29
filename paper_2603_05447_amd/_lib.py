"""ctypes declarations for libgpe.so (the C ABI in include/gpe.h)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgpe.so")

GPE_OK, GPE_ERR_ARG, GPE_ERR_ALLOC, GPE_ERR_DEVICE, GPE_ERR_STATE, GPE_ERR_UNSTABLE, GPE_ERR_NONFINITE = range(7)
STATUS_NAMES = ["GPE_OK", "GPE_ERR_ARG", "GPE_ERR_ALLOC", "GPE_ERR_DEVICE", "GPE_ERR_STATE",
                "GPE_ERR_UNSTABLE", "GPE_ERR_NONFINITE"]
GPE_C128, GPE_C64 = 0, 1
GPE_MODE_ITP, GPE_MODE_RT, GPE_MODE_ADJ, GPE_MODE_RT_RKHE3, GPE_MODE_RT_RKCK, GPE_MODE_ITP_REAL = range(6)
GPE_RK4, GPE_RKHE3, GPE_RKCK = 0, 1, 2
GPE_POT_STATIC, GPE_POT_RF_RAMP, GPE_POT_LERP, GPE_POT_SHELL_RAMP = 0, 1, 2, 3
GPE_MAX_KNOTS = 32


class Geometry(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("h", C.c_double * 3), ("x0", C.c_double * 3)]


class Potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_knots", C.c_int32), ("field", C.c_void_p), ("omega", C.c_double),
                ("knot_t", C.POINTER(C.c_double)), ("knot_delta", C.POINTER(C.c_double)), ("field2", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("dt", C.c_double), ("norm_target", C.c_double), ("obs_every", C.c_int64),
                ("skip_stability_check", C.c_int32), ("integrator", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("norm", C.c_double), ("energy", C.c_double), ("mu", C.c_double)]


class Ramp(C.Structure):
    _fields_ = [("omega", C.c_double), ("n_knots", C.c_int32), ("kind", C.c_int32),
                ("knot_t", C.POINTER(C.c_double)), ("knot_delta", C.POINTER(C.c_double))]


_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_pd = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "gpe_last_error": (C.c_char_p, []),
    "gpe_abi_version": (C.c_int, []),
    "gpe_grid_create": (C.c_int, [C.POINTER(Geometry), _vp, C.c_int, C.POINTER(_vp)]),
    "gpe_grid_create_runs": (C.c_int, [C.POINTER(Geometry), _i64, _vp, C.c_int, C.POINTER(_vp)]),
    "gpe_grid_create_threshold": (C.c_int, [C.POINTER(Geometry), C.c_int, _vp, _vp, C.c_double, C.c_int,
                                            C.POINTER(_vp)]),
    "gpe_remap": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _vp]),
    "gpe_grid_info": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "gpe_grid_segments": (C.c_int, [_vp, _vp]),
    "gpe_grid_runs": (C.c_int, [_vp, _vp]),
    "gpe_grid_set_stencil": (C.c_int, [_vp, _i32]),
    "gpe_grid_get_stencil": (C.c_int, [_vp, C.POINTER(_i32)]),
    "gpe_grid_stencil_segments": (C.c_int, [_vp, _i32, C.POINTER(_i64), _vp]),
    "gpe_grid_destroy": (C.c_int, [_vp]),
    "gpe_work_bytes": (C.c_int, [_vp, C.c_int, _i32, _i64, _i64, C.POINTER(C.c_size_t)]),
    "gpe_pack": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "gpe_unpack": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "gpe_pack_real": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "gpe_imag_time": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(Potential), C.POINTER(Params), _i64, _vp,
                                C.c_size_t, _vp, C.POINTER(Obs), _vp]),
    "gpe_imag_time_real": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(Potential), C.POINTER(Params), _i64, _vp,
                                     C.c_size_t, _vp, C.POINTER(Obs), _vp]),
    "gpe_real_time": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(Potential), C.POINTER(Params), C.c_double, _i64,
                                _vp, C.c_size_t, _vp, C.POINTER(Obs), _vp]),
    "gpe_real_time_noalloc": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(Potential), C.POINTER(Params), C.c_double,
                                        _i64, _vp, C.POINTER(Obs), _vp]),
    "gpe_noalloc_scratch_bytes": (C.c_size_t, []),
    "gpe_observe": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(Potential), C.c_double, C.c_double, _vp,
                              C.POINTER(Obs)]),
    "gpe_overlap": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _pd]),
    "gpe_fidelity_grad": (C.c_int, [_vp, C.c_int, _vp, _vp, C.POINTER(Potential), C.POINTER(Params), C.c_double,
                                    _i64, _i64, _vp, C.c_size_t, _vp, _pd, _pd, _vp]),
    "gpe_staged_ramp_grids": (C.c_int, [C.POINTER(Geometry), C.c_int, _i32, C.POINTER(_vp), _pd, C.c_double,
                                        C.c_int, C.POINTER(_vp), _pd]),
    "gpe_staged_ramp_work_bytes": (C.c_int, [_i32, C.POINTER(_vp), C.c_int, _i32, C.POINTER(C.c_size_t)]),
    "gpe_staged_ramp_run": (C.c_int, [_vp, _vp, _i32, C.POINTER(_vp), C.POINTER(_vp), C.c_int, C.POINTER(_vp),
                                      C.POINTER(Params), C.c_double, _i64, _vp, C.c_size_t, _vp, _pd]),
    "gpe_batch_create": (C.c_int, [_i32, C.POINTER(_vp), C.c_int, C.POINTER(_vp)]),
    "gpe_batch_offsets": (C.c_int, [_vp, C.POINTER(_i64)]),
    "gpe_batch_destroy": (C.c_int, [_vp]),
    "gpe_batch_work_bytes": (C.c_int, [_vp, C.c_int, _i32, _i64, _i64, C.POINTER(C.c_size_t)]),
    "gpe_batch_real_time": (C.c_int, [_vp, C.c_int, _vp, _vp, C.POINTER(Ramp), C.POINTER(Params), C.c_double,
                                      _i64, _i32, _vp, C.c_size_t, _vp, C.POINTER(Obs)]),
    "gpe_batch_fidelity_grad": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, C.POINTER(Ramp), C.POINTER(Params),
                                          C.c_double, _i64, _i64, _i32, _vp, C.c_size_t, _vp, _pd, _pd]),
    "gpe_config_count": (_i32, []),
    "gpe_config_describe": (C.c_int, [_i32] + [C.POINTER(_i32)] * 6),
    "gpe_grid_set_config": (C.c_int, [_vp, _i32]),
    "gpe_grid_get_config": (C.c_int, [_vp, C.POINTER(_i32)]),
    "gpe_batch_set_config": (C.c_int, [_vp, _i32]),
    "gpe_batch_get_config": (C.c_int, [_vp, C.POINTER(_i32)]),
    "gpe_batch_autotune": (C.c_int, [_vp, C.c_int, _vp, _vp, C.POINTER(Ramp), C.POINTER(Params), _i32, _i32, _vp,
                                     C.c_size_t, _vp, C.POINTER(_i32), _pd]),
    "gpe_batch_apply_tuned": (C.c_int, [_vp, C.c_int, C.POINTER(_i32)]),
    "gpe_grid_autotune": (C.c_int, [_vp, C.c_int, _i32, _vp, C.POINTER(Potential), C.POINTER(Params), _i32, _vp,
                                    C.c_size_t, _vp, C.POINTER(_i32), _pd]),
    "gpe_grid_apply_tuned": (C.c_int, [_vp, C.c_int, _i32, C.POINTER(_i32)]),
    "gpe_autotune_cache_clear": (C.c_int, []),
    "gpe_timing_enable": (C.c_int, [_i32]),
    "gpe_timing_reset": (C.c_int, []),
    "gpe_timing_count": (_i32, []),
    "gpe_timing_name": (C.c_char_p, [_i32]),
    "gpe_timing_read": (C.c_int, [_i32, C.POINTER(_i64), _pd]),
    "gpe_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
}

_lib = None


def load() -> C.CDLL:
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_05447_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class GPEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


def check(status: int) -> None:
    if status != GPE_OK:
        raise GPEError(status, load().gpe_last_error().decode(errors="replace"))
