"""ctypes declarations of the C ABI in include/dwt2.h.

The library is loaded from this package directory only. If it is missing the
load fails loudly: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdwt2.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = 0, -1, -2, -3, -4
CDF97, CDF53 = 0, 1
EXT_WHOLE_SAMPLE_SYMMETRIC = 0
F32, F16, BF16 = 0, 1, 2
NONSEPARABLE, SEPARABLE, NONSEPARABLE_LDS, SEPARABLE_LDS = 0, 1, 2, 3
TILE_TAIL = -2            # tiles[j] of a level that runs in the fused tail launch
TILE_HEAD = -3            # tiles[0] and tiles[1]: levels 1 and 2 in one fused launch
TAIL_MAX = 3
TAIL_AUTO_PIXELS = 1 << 22
STATIC_WORKSPACE_BYTES = 64 << 20   # DWT2_STATIC_WORKSPACE_BYTES

# Every function declared in include/dwt2.h: name -> (restype, argtypes)
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_ip32 = ctypes.POINTER(ctypes.c_int32)


class Desc(ctypes.Structure):
    """dwt2_desc."""
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch", ctypes.c_int64), ("dtype", ctypes.c_int32)]


_DescP = ctypes.POINTER(Desc)


class Image(ctypes.Structure):
    """dwt2_image: one image of a batch."""
    _fields_ = [("src", ctypes.c_void_p), ("src_pitch", ctypes.c_int64),
                ("dst", ctypes.c_void_p), ("dst_pitch", ctypes.c_int64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_ImageP = ctypes.POINTER(Image)


class LevelJob(ctypes.Structure):
    """dwt2_level_job: one level of one image."""
    _fields_ = [("full", ctypes.c_void_p), ("full_pitch", ctypes.c_int64),
                ("full_dtype", ctypes.c_int32),
                ("ll", ctypes.c_void_p), ("ll_pitch", ctypes.c_int64),
                ("ll_dtype", ctypes.c_int32),
                ("hl", ctypes.c_void_p), ("lh", ctypes.c_void_p), ("hh", ctypes.c_void_p),
                ("band_pitch", ctypes.c_int64), ("band_dtype", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_LevelJobP = ctypes.POINTER(LevelJob)
SIZE_CLASSES = 4
BATCH_PERSISTENT = 1      # DWT2_BATCH_PERSISTENT
PLAN_HEAD = 1             # DWT2_PLAN_HEAD: levels 1 and 2 of a batch in one head launch

SIGNATURES = {
    "dwt2_workspace_bytes": (_sz, [_i32, _i32, _i32, _i32]),
    # src, src_d, coef, coef_d, wavelet, levels, boundary, scheme, workspace, bytes, stream
    "dwt2_forward": (ctypes.c_int, [_vp, _DescP, _vp, _DescP, _i32, _i32, _i32, _i32,
                                    _vp, _sz, _vp]),
    "dwt2_inverse": (ctypes.c_int, [_vp, _DescP, _vp, _DescP, _i32, _i32, _i32, _i32,
                                    _vp, _sz, _vp]),
    # ... plus tiles and level events before the stream
    "dwt2_forward_ex": (ctypes.c_int, [_vp, _DescP, _vp, _DescP, _i32, _i32, _i32, _i32,
                                       _vp, _sz, _ip32, _vp, _vp]),
    "dwt2_inverse_ex": (ctypes.c_int, [_vp, _DescP, _vp, _DescP, _i32, _i32, _i32, _i32,
                                       _vp, _sz, _ip32, _vp, _vp]),
    "dwt2_forward_no_alloc": (ctypes.c_int, [_vp, _DescP, _vp, _DescP, _i32, _i32, _i32, _i32,
                                             _vp]),
    "dwt2_forward_level": (ctypes.c_int, [_vp, _i64, _i32, _i32, _i32, _vp, _i64, _i32,
                                          _vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp]),
    "dwt2_inverse_level": (ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _i64, _i32,
                                          _vp, _i64, _i32, _i32, _i32, _i32, _i32, _i32, _vp]),
    "dwt2_tile_config_count": (ctypes.c_int, []),
    "dwt2_tile_config_info": (ctypes.c_int, [_i32, _i32, _ip32, _ip32, _ip32, _ip32, _ip32]),
    "dwt2_default_tile": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32]),
    "dwt2_size_class": (ctypes.c_int, [_i32, _i32]),
    "dwt2_batch_plan_bytes": (ctypes.c_int, [_ImageP, _i32, _i32, _i32, _i32, _i32, _i32,
                                             _ip32, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "dwt2_batch_plan": (ctypes.c_int, [_ImageP, _i32, _i32, _i32, _i32, _i32, _i32, _ip32,
                                       _i32, _vp, _sz]),
    "dwt2_batch_launches": (ctypes.c_int, [_vp, _sz, _ip32, _ip32]),
    "dwt2_batch_run": (ctypes.c_int, [_vp, _sz, _vp, _i32, _i32, _vp]),
    "dwt2_forward_level_batch": (ctypes.c_int, [_LevelJobP, _i32, _i32, _i32, _ip32, _vp]),
    "dwt2_inverse_level_batch": (ctypes.c_int, [_LevelJobP, _i32, _i32, _i32, _ip32, _vp]),
    "dwt2_forward_head_batch": (ctypes.c_int, [_LevelJobP, _i32, _i32, _i32, _vp]),
    "dwt2_inverse_head_batch": (ctypes.c_int, [_LevelJobP, _i32, _i32, _i32, _vp]),
    "dwt2_fused_levels": (ctypes.c_int, [_i32, _i32, _i32]),
    "dwt2_head_levels": (ctypes.c_int, [_i32, _i32, _i32]),
    "dwt2_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dwt2_last_hip_error": (ctypes.c_int, []),
    "dwt2_version": (ctypes.c_int, []),
}

_lib = None


class DWT2Error(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        text = load().dwt2_status_string(status).decode()
        extra = ""
        if status == ERR_HIP:
            extra = f" (hipError_t {load().dwt2_last_hip_error()})"
        super().__init__(f"{what}: {text}{extra}" if what else text + extra)


def load():
    """Load libdwt2.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run paper_1705_08266_amd.build.build() "
            "(hipcc --offload-arch=gfx950). There is no fallback path.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str = ""):
    if status != OK:
        raise DWT2Error(status, what)
