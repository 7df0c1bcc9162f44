"""ctypes binding of libxs.so (the C ABI declared in include/xs.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If libxs.so is missing, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxs.so")

XS_OK, XS_EINVAL, XS_ENOMEM, XS_EDEVICE, XS_ENOTSUP = 0, 1, 2, 3, 4
XS_FP64, XS_FP32C = 0, 1
STATUS_NAMES = {0: "XS_OK", 1: "XS_EINVAL", 2: "XS_ENOMEM", 3: "XS_EDEVICE", 4: "XS_ENOTSUP"}

EXPORTS = [
    "xs_intensity_direct", "xs_intensity_grad", "xs_g2_rings", "xs_xsvs_contrast",
    "xs_last_error", "xs_version", "xs_shutdown", "xs_get_tile_shape", "xs_set_tile_shape",
    "xs_speckle_loss", "xs_position_step", "xs_timing_enable", "xs_timing_read",
    "xs_roofline_probe", "xs_plan_create", "xs_plan_intensity", "xs_plan_grad", "xs_plan_destroy",
    "xs_plan_describe", "xs_isf_rings", "xs_siegert", "xs_intensity_species", "xs_intensity_species_grad",
    "xs_frame_sums", "xs_ring_histogram", "xs_plan_create_species", "xs_plan_intensity_species",
    "xs_plan_grad_species", "xs_g2_rings_noalloc", "xs_fft_intensity", "xs_plan_create_forward",
]

_P = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class XsBatch(ctypes.Structure):
    _fields_ = [
        ("n_sys", ctypes.c_int32),
        ("n_atoms", _i64p),
        ("n_q", _i64p),
        ("n_frames", _i32p),
        ("pos_off", _i64p),
        ("f_off", _i64p),
        ("q_off", _i64p),
        ("out_off", _i64p),
        ("box", _dp),
    ]


class XsTileShape(ctypes.Structure):
    _fields_ = [
        ("atoms_per_tile", ctypes.c_int32),
        ("q_per_lane", ctypes.c_int32),
        ("atom_split", ctypes.c_int32),
        ("pixel_split", ctypes.c_int32),
        ("waves_per_simd", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
    ]


class XsPlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_segments", ctypes.c_int32),
        ("n_lattice_segments", ctypes.c_int32),
        ("n_forward_items", ctypes.c_int32),
        ("n_gradient_items", ctypes.c_int32),
        ("device_bytes", ctypes.c_int64),
        ("n_row_segments", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class XsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


_lib = None


def load():
    """Load libxs.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libxs.so is not built (%s); run __graft_entry__.build() or "
            "python -m paper_2204_13241_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i32 = ctypes.c_int32
    i64 = ctypes.c_int64
    bp = ctypes.POINTER(XsBatch)
    sp = ctypes.POINTER(XsTileShape)
    sig = {
        "xs_intensity_direct": (i32, [bp, _P, _P, _P, i32, _P, _P, _P]),
        "xs_intensity_grad": (i32, [bp, _P, _P, _P, _P, _P, i32, _P, _P, _P]),
        "xs_g2_rings": (i32, [_P, i64, i64, _P, _P, i32, i32, _P, _P, _P]),
        "xs_g2_rings_noalloc": (i32, [_P, i64, i64, _P, _P, i32, i32, _P, _P, _P]),
        "xs_fft_intensity": (i32, [_P, _P, i64, ctypes.c_double, i32, ctypes.c_double, i32, _P, _P, _P]),
        "xs_xsvs_contrast": (i32, [_P, i64, i64, _P, _P, i32, i32, _P, _P, _P]),
        "xs_isf_rings": (i32, [_P, i64, i64, _P, _P, i32, i32, ctypes.c_double, _P, _P, _P]),
        "xs_siegert": (i32, [_P, _P, i32, i32, i32, _P, _P, _P, _P]),
        "xs_intensity_species": (i32, [bp, _P, _P, i32, _P, _P, i32, _P, _P, _P]),
        "xs_intensity_species_grad": (i32, [bp, _P, _P, i32, _P, _P, _P, _P, i32, _P, _P, _P]),
        "xs_frame_sums": (i32, [_P, i64, i64, i64, i64, i64, i64, ctypes.c_double, _P, _P]),
        "xs_ring_histogram": (i32, [_P, i64, i64, _P, _P, i32, i32, ctypes.c_double, _P, _P, _P]),
        "xs_last_error": (ctypes.c_char_p, []),
        "xs_version": (i32, []),
        "xs_shutdown": (i32, []),
        "xs_get_tile_shape": (i32, [i32, sp]),
        "xs_set_tile_shape": (i32, [i32, sp]),
        "xs_speckle_loss": (i32, [_P, _P, i64, _P, _P, _P]),
        "xs_position_step": (i32, [_P, _P, _P, i64, ctypes.c_double, _P]),
        "xs_timing_enable": (i32, [i32]),
        "xs_timing_read": (i32, [i32, _dp, _i64p, _dp]),
        "xs_roofline_probe": (i32, [i32, i64, _dp, _P]),
        "xs_plan_create": (i32, [bp, _P, ctypes.POINTER(_P), _P]),
        "xs_plan_create_forward": (i32, [bp, _P, ctypes.POINTER(_P), _P]),
        "xs_plan_intensity": (i32, [_P, _P, _P, _P, _P, _P]),
        "xs_plan_grad": (i32, [_P, _P, _P, _P, _P, i32, _P, _P, _P]),
        "xs_plan_create_species": (i32, [bp, _P, _P, i32, _P, ctypes.POINTER(_P), _P]),
        "xs_plan_intensity_species": (i32, [_P, _P, _P, _P, _P]),
        "xs_plan_grad_species": (i32, [_P, _P, _P, _P, i32, _P, _P, _P]),
        "xs_plan_destroy": (i32, [_P]),
        "xs_plan_describe": (i32, [_P, ctypes.POINTER(XsPlanInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != XS_OK:
        msg = load().xs_last_error()
        raise XsError(status, msg.decode() if msg else "")
