"""ctypes declarations of the C ABI in include/gs3tr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_uint8, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgs3tr.so")

GS3_OK = 0
GS3_EINVAL = -1
GS3_ENOMEM = -2
GS3_EDEVICE = -3
GS3_ENONFINITE = -4
GS3_ESTATE = -5
GS3_ENOTIMPL = -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE", -5: "ESTATE", -6: "ENOTIMPL"}


class Camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("R", c_float * 9), ("t", c_float * 3)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_gaussians", c_int64), ("sh_degree", c_int32), ("n_cameras", c_int32),
                ("cameras", POINTER(Camera)), ("background", c_float * 3), ("lambda_dssim", c_float),
                ("flags", c_uint32), ("train_mask", POINTER(c_uint8))]


class TrHparams(ctypes.Structure):
    _fields_ = [("theta1", c_float), ("theta2", c_float), ("epsilon", c_float), ("variant", c_uint32)]


class GS3Error(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_SIGS = {
    "gs3_n_params": (c_int32, [c_int32]),
    "gs3_version": (c_char_p, []),
    "gs3_last_error": (c_char_p, []),
    "gs3_scene_create": (c_int32, [POINTER(SceneDesc), c_void_p, c_void_p, c_void_p, POINTER(c_void_p)]),
    "gs3_scene_destroy": (c_int32, [c_void_p]),
    "gs3_scene_params": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "gs3_scene_set_params": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "gs3_scene_bytes": (c_int32, [POINTER(SceneDesc), POINTER(c_int64), POINTER(c_int64)]),
    "gs3_scene_device_bytes": (c_int32, [c_void_p, POINTER(c_int64)]),
    "gs3_trim_cache": (c_int32, []),
    "gs3_scene_sync": (c_int32, [c_void_p]),
    "gs3_render": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "gs3_render_noalloc": (c_int32, [c_int64, c_int32, c_void_p, POINTER(Camera), POINTER(c_float), c_void_p,
                                     c_void_p]),
    "gs3_bin": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int64, POINTER(c_int64), c_void_p]),
    "gs3_grad": (c_int32, [c_void_p, POINTER(c_int32), c_int32, c_void_p, POINTER(c_double), c_void_p]),
    "gs3_hvp_diag": (c_int32, [c_void_p, POINTER(c_int32), c_int32, c_int32, c_uint64, c_void_p, c_void_p]),
    "gs3_tr_step": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(TrHparams), c_void_p, c_void_p, c_void_p]),
    "gs3_tr_iteration": (c_int32, [c_void_p, POINTER(c_int32), c_int32, POINTER(c_int32), c_int32, c_int32, c_uint64,
                                   POINTER(TrHparams), POINTER(c_double), c_void_p]),
    "gs3_adam_step": (c_int32, [c_void_p, c_void_p, POINTER(c_float), c_int32, c_void_p]),
    "gs3_adam_tr_step": (c_int32, [c_void_p, c_void_p, POINTER(c_float), c_int32, c_float, c_void_p]),
    "gs3_psnr": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_void_p]),
    "gs3_render_vjp": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "gs3_render_jvp": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs3_scene_export": (c_int32, [c_void_p] + [c_void_p] * 5 + [c_void_p]),
    "gs3_scene_import": (c_int32, [c_void_p] + [c_void_p] * 5 + [c_void_p]),
    "gs3_profile_enable": (c_int32, [c_char_p]),
    "gs3_profile_count": (c_int32, [c_int32]),
    "gs3_profile_read": (c_int32, [c_char_p, POINTER(c_int64), POINTER(c_double), POINTER(c_int64),
                                   POINTER(c_int64)]),
    "gs3_profile_reset": (c_int32, []),
}

_lib = None


def load():
    """Load libgs3tr.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2602_00395_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn_name: str, code: int):
    if code != GS3_OK:
        msg = _lib.gs3_last_error().decode() if _lib is not None else ""
        raise GS3Error(fn_name, code, msg)


def declared_functions(header_path: str) -> list:
    """Names of the functions declared in include/gs3tr.h."""
    import re

    text = open(header_path).read()
    return sorted(set(re.findall(r"^\s*(?:gs3_status|int32_t|const char\*)\s+(gs3_\w+)\s*\(", text, re.M)))
