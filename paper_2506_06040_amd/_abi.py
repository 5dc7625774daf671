"""ctypes view of include/ntc.h and loader of libntc.so.

Only argument marshalling lives here; every step of the decode runs in the
HIP kernels of libntc.so. There is no fallback: if the library is missing
or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libntc.so")

MAX_LEVELS = 4
MAX_LAYERS = 5

# ntc_status
OK, E_NULL, E_SHAPE, E_UNSUPPORTED, E_WORKSPACE, E_HIP, E_ALIGN = range(7)
# ntc_dtype
F32, F16, BF16, FP8_E4M3 = 0, 1, 2, 3
# ntc_latent_fmt
LATENT_BC1, LATENT_F32 = 0, 1
# ntc_address
CLAMP, WRAP = 0, 1


class NtcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class ntc_latents(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("format", ctypes.c_int32),
                ("address", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("width", ctypes.c_int32 * MAX_LEVELS), ("height", ctypes.c_int32 * MAX_LEVELS),
                ("shift", (ctypes.c_float * 2) * MAX_LEVELS),
                ("data", ctypes.c_void_p * MAX_LEVELS)]


class ntc_mlp(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("dims", ctypes.c_int32 * (MAX_LAYERS + 1)),
                ("W", ctypes.c_void_p * MAX_LAYERS), ("b", ctypes.c_void_p * MAX_LAYERS)]


class ntc_tile_cfg(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("tiles_per_iter", ctypes.c_int32),
                ("stage_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ntc_material(ctypes.Structure):
    _fields_ = [("lat", ntc_latents), ("mlp", ntc_mlp), ("packed", ctypes.c_void_p),
                ("uv", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", ctypes.c_void_p),
                ("out_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pixel_index", ctypes.c_void_p), ("image_pixels", ctypes.c_int64)]


class ntc_batch_cfg(ctypes.Structure):
    _fields_ = [("item_pixels", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("stage_capacity", ctypes.c_int32), ("n_cus", ctypes.c_int32)]


MAX_MIPS = 12
FILTER_TRILINEAR, FILTER_ANISOTROPIC = 1, 2


class ntc_latent_mips(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_mips", ctypes.c_int32 * MAX_LEVELS),
                ("width", ctypes.c_int32 * MAX_LEVELS), ("height", ctypes.c_int32 * MAX_LEVELS),
                ("shift", (ctypes.c_float * 2) * MAX_LEVELS),
                ("data", (ctypes.c_void_p * MAX_MIPS) * MAX_LEVELS)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); the exported C ABI, in header order
SIGNATURES = {
    "ntc_status_string": (ctypes.c_char_p, [_I32]),
    "ntc_last_error": (ctypes.c_char_p, []),
    "ntc_version": (_I32, []),
    "ntc_mlp_pack_size": (_I32, [ctypes.POINTER(ntc_mlp), _I32, ctypes.POINTER(_SZ)]),
    "ntc_mlp_pack": (_I32, [ctypes.POINTER(ntc_mlp), _I32, _P, _P, _SZ, _P]),
    "ntc_calibrate_fp8": (_I32, [ctypes.POINTER(ntc_latents), ctypes.POINTER(ntc_mlp), _P, _P, _I64, _P, _P]),
    "ntc_decode": (_I32, [ctypes.POINTER(ntc_latents), ctypes.POINTER(ntc_mlp), _I32, _P, _P, _I64, _P, _I32,
                          ctypes.POINTER(ntc_tile_cfg), _P]),
    "ntc_decode_backward_workspace": (_I32, [ctypes.POINTER(ntc_latents), ctypes.POINTER(ntc_mlp), _I64,
                                             ctypes.POINTER(_SZ)]),
    "ntc_decode_backward": (_I32, [ctypes.POINTER(ntc_latents), ctypes.POINTER(ntc_mlp), _P, _I64, _P,
                                   ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _SZ, _P]),
    "ntc_decode_filtered": (_I32, [ctypes.POINTER(ntc_latent_mips), ctypes.POINTER(ntc_mlp), _P, _P, _P, _I64, _P,
                                   _I32, _I32, _I32, _P]),
    "ntc_qat_texels": (_I32, [_P, _I32, _I32, _P, _P]),
    "ntc_qat_backward": (_I32, [_P, _I32, _I32, _P, _P, _P]),
    "ntc_qat_export_bc1": (_I32, [_P, _I32, _I32, _P, _P]),
    "ntc_classify_workspace": (_I32, [_I32, _I32, _I32, ctypes.POINTER(_SZ)]),
    "ntc_classify": (_I32, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "ntc_classify_noalloc": (_I32, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P]),
    "ntc_gather_uv": (_I32, [_P, _P, _I64, _P, _P]),
    "ntc_scatter_rows": (_I32, [_P, _P, _I64, _I32, _I32, _P, _P]),
    "ntc_batched_plan_size": (_I32, [ctypes.POINTER(ntc_material), _I32, ctypes.POINTER(ntc_batch_cfg),
                                     ctypes.POINTER(_SZ)]),
    "ntc_batched_plan": (_I32, [ctypes.POINTER(ntc_material), _I32, ctypes.POINTER(ntc_batch_cfg), _P, _SZ]),
    "ntc_decode_batched": (_I32, [_P, _P, _SZ, _P]),
    "ntc_bc1_decode_texels": (_I32, [ctypes.POINTER(ntc_latents), _I32, _P, _P, _P]),
}

_lib = None


def lib():
    """The loaded libntc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NtcError(E_HIP, f"libntc.so is not built ({LIB_PATH}); build it with python paper_2506_06040_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    """Raise NtcError for a status other than NTC_OK."""
    if status != OK:
        L = lib()
        detail = L.ntc_last_error().decode()
        name = L.ntc_status_string(status).decode()
        raise NtcError(status, f"{name}: {detail}")
