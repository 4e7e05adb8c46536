"""ctypes declarations of the C ABI in include/aw.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaw.so")

AW_OK, AW_EINVAL, AW_EUNSUPPORTED, AW_EDEVICE, AW_ENOMEM, AW_EWORKSPACE = range(6)
STATUS_NAMES = {0: "AW_OK", 1: "AW_EINVAL", 2: "AW_EUNSUPPORTED", 3: "AW_EDEVICE", 4: "AW_ENOMEM",
                5: "AW_EWORKSPACE"}
MAP_STDMAP, MAP_S2, MAP_S4, MAP_S6, MAP_Y6 = 1, 2, 4, 6, 7
IC_GRID2, IC_BOX, IC_EXPLICIT, IC_SPHERE, IC_CLOUD = 0, 1, 2, 3, 4
F_TANGENT = 1
F_WINDOW = 2
OUT_L, OUT_LAMBDA, OUT_CHI, OUT_VX, OUT_VY, OUT_VZ, OUT_DP2, OUT_J, OUT_DE, NOUT = range(10)
NCARRY = 22
IMG_IC_GRID, IMG_HIST_P0, IMG_HIST_VDIR = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTS = [
    "aw_last_error", "aw_version", "aw_release", "aw_ensemble_size", "aw_generate_ic",
    "aw_map_ensemble", "aw_map_ensemble_steps", "aw_indicator_image", "aw_window_density", "aw_histogram2d", "aw_histogram2d_noalloc",
    "aw_vdir_keys", "aw_image_workspace", "aw_reserve", "aw_indicator_grad_workspace", "aw_indicator_grad", "aw_indicator_grad_reversible",
    "aw_indicator_grad_reversible_workspace", "aw_ftle_grad_reversible_workspace",
    "aw_ftle_grad_workspace", "aw_ftle_grad", "aw_ftle_grad_reversible",
    "aw_graph_create",
    "aw_graph_launch", "aw_graph_destroy", "aw_timing_enable", "aw_timing_read",
    "aw_step_op_counts",
]


class AwEnsemble(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32),
        ("map_form", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("h", ctypes.c_double),
        ("n_steps", ctypes.c_int64),
        ("ic_kind", ctypes.c_int32),
        ("axis", ctypes.c_int32 * 2),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("base", ctypes.c_double * 6),
        ("box_lo", ctypes.c_double * 6),
        ("box_hi", ctypes.c_double * 6),
        ("n_orbits", ctypes.c_int64),
        ("seed_ic", ctypes.c_uint64),
        ("seed_tangent", ctypes.c_uint64),
        ("chi_threshold", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("energy", ctypes.c_double),
        ("window", ctypes.c_double * 4),
        ("cloud", ctypes.c_double * 4),
    ]


class AwTuning(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("orbits_per_lane", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("renorm_every", ctypes.c_int32),
        ("persistent_wgs", ctypes.c_int32),
        ("lanes_per_orbit", ctypes.c_int32),
    ]


class AwImageSpec(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("field", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("key_axis", ctypes.c_int32 * 2),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
    ]


_vp = ctypes.c_void_p
_i32, _i64, _f64, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
_PE = ctypes.POINTER(AwEnsemble)
_PT = ctypes.POINTER(AwTuning)
_PS = ctypes.POINTER(AwImageSpec)
_PP = ctypes.POINTER(ctypes.c_void_p)

SIGNATURES = {
    "aw_last_error": (ctypes.c_char_p, []),
    "aw_version": (ctypes.c_char_p, []),
    "aw_release": (_i32, []),
    "aw_ensemble_size": (_i64, [_PE]),
    "aw_generate_ic": (_i32, [_PE, _vp, _vp, _vp, _vp]),
    "aw_map_ensemble": (_i32, [_PE, _i32, _PP, _PP, _PP, _PP, _PT, _vp]),
    "aw_map_ensemble_steps": (_i32, [_PE, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _PT, _vp]),
    "aw_indicator_image": (_i32, [_PE, _i32, _PS, _PP, _PP, _PP, _PT, _vp]),
    "aw_window_density": (_i32, [_PE, _vp, _vp, _i64, _i64, _i64, _PS, _vp, _PT, _vp]),
    "aw_histogram2d": (_i32, [_i64, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "aw_histogram2d_noalloc": (_i32, [_i64, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _i32, _i32, _i32, _vp, _vp, _vp,
                                      _vp]),
    "aw_vdir_keys": (_i32, [_i64, _vp, _vp, _vp, _vp]),
    "aw_image_workspace": (_i32, [_PE, _i32, _PS, ctypes.POINTER(ctypes.c_size_t)]),
    "aw_reserve": (_i32, [ctypes.c_size_t, _vp]),
    "aw_indicator_grad_workspace": (_i32, [_PE, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "aw_indicator_grad": (_i32, [_PE, _vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _PT, _vp]),
    "aw_indicator_grad_reversible": (_i32, [_PE, _vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _PT, _vp]),
    "aw_ftle_grad_workspace": (_i32, [_PE, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "aw_indicator_grad_reversible_workspace": (_i32, [_PE, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "aw_ftle_grad_reversible_workspace": (_i32, [_PE, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "aw_ftle_grad": (_i32, [_PE, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _PT, _vp]),
    "aw_ftle_grad_reversible": (_i32, [_PE, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _PT, _vp]),
    "aw_graph_create": (_i32, [_PE, _i32, _PS, _PP, _PP, _PP, _PT, ctypes.POINTER(_vp)]),
    "aw_graph_launch": (_i32, [_vp, _vp]),
    "aw_graph_destroy": (None, [_vp]),
    "aw_timing_enable": (_i32, [_i32]),
    "aw_timing_read": (_i32, [ctypes.POINTER(_f64), ctypes.POINTER(_i64)]),
    "aw_step_op_counts": (_i32, [_i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
}

_lib = None


class AwError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load():
    """Load libaw.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1107_4107_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != AW_OK:
        raise AwError(status, load().aw_last_error().decode())


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
    return arr
