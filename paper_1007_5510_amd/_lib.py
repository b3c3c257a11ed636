"""ctypes view of the C ABI in include/rpca.h (argument marshalling only).

The library is the in-tree ``librpca.so`` built by ``paper_1007_5510_amd.build``.
torch is imported first so that the library binds to the HIP runtime torch
already loaded (same soname); nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpca.so")

RPCA_OK = 0
STATUS_NAMES = {
    0: "RPCA_OK", 1: "RPCA_ERR_INVALID_ARG", 2: "RPCA_ERR_UNSUPPORTED", 3: "RPCA_ERR_OUT_OF_MEMORY",
    4: "RPCA_ERR_HIP", 5: "RPCA_ERR_CALLBACK", 6: "RPCA_ERR_NONFINITE", 7: "RPCA_ERR_QR_BREAKDOWN",
    8: "RPCA_ERR_NO_STATE", 9: "RPCA_ERR_SCRATCH_LIMIT",
}
STORAGE = {"f32": 0, "bf16": 1, "fp8_e4m3": 2, "bf16_hilo": 3}
SOURCE = {"device": 0, "host_pinned": 1, "callback": 2, "device_callback": 3}
FLAG_KEEP_STATE = 1 << 0
FLAG_PROFILE = 1 << 1
FLAG_FORCE_FALLBACK = 1 << 2
FLAG_NO_RESCALE = 1 << 3
FLAG_SPLIT_BF16 = 1 << 4
FLAG_FP64_STEP1 = 1 << 5
FLAG_FORCE_HOUSEHOLDER = 1 << 6
FLAG_FUSED = 1 << 7
STATE = {"H": 0, "HSCALE": 1, "Q": 2, "T": 3, "SIGMA": 4, "W": 5, "MU": 6, "H64": 7}


class Desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64),
        ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("i", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("source", ctypes.c_int32), ("center", ctypes.c_int32),
        ("panel_rows", ctypes.c_int64), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
        ("device", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("ms_total", ctypes.c_double), ("ms_colmean", ctypes.c_double), ("ms_power", ctypes.c_double),
        ("ms_qr", ctypes.c_double), ("ms_tpass", ctypes.c_double), ("ms_small_svd", ctypes.c_double),
        ("ms_assemble", ctypes.c_double), ("ms_fwd_kernel", ctypes.c_double), ("ms_adj_kernel", ctypes.c_double),
        ("fwd_launches", ctypes.c_int64), ("adj_launches", ctypes.c_int64), ("a_bytes_read", ctypes.c_int64),
        ("h2d_bytes", ctypes.c_int64), ("qr_fallback", ctypes.c_int32), ("eig_vectors", ctypes.c_int32),
        ("hip_error", ctypes.c_int32), ("passes", ctypes.c_int32),
        ("ms_tpass_kernel", ctypes.c_double), ("tpass_launches", ctypes.c_int64),
        ("a_reads", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("ms_fused_kernel", ctypes.c_double), ("fused_launches", ctypes.c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


PANEL_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                            ctypes.c_int64, ctypes.c_void_p)

DEVICE_PANEL_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_void_p)

_lib = None


def load(path: str = LIB_PATH):
    """Load librpca.so; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1007_5510_amd.build`")
    try:
        import torch  # noqa: F401  (binds the HIP runtime torch ships, same soname)
    except Exception:
        pass
    lib = ctypes.CDLL(path)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.rpca_plan.argtypes = [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]
    lib.rpca_plan.restype = i32
    lib.rpca_factor.argtypes = [vp, vp, i64, vp, PANEL_CB, vp, vp, vp, i64, vp, vp, i64]
    lib.rpca_factor.restype = i32
    lib.rpca_backward.argtypes = [vp, vp, vp, i64, vp, i64, vp, i64]
    lib.rpca_backward.restype = i32
    lib.rpca_residual.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, i64, i32, i32, u64,
                                  ctypes.POINTER(ctypes.c_double)]
    lib.rpca_residual.restype = i32
    lib.rpca_quantize.argtypes = [i32, i64, i64, vp, i64, vp, i64, vp, vp, i32, vp]
    lib.rpca_quantize.restype = i32
    lib.rpca_quantize_noalloc.argtypes = [i32, i64, i64, vp, i64, vp, i64, vp, vp, i32, vp]
    lib.rpca_quantize_noalloc.restype = i32
    lib.rpca_get_state.argtypes = [vp, i32, vp, i64]
    lib.rpca_get_state.restype = i32
    lib.rpca_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.rpca_get_stats.restype = i32
    lib.rpca_status_str.argtypes = [i32]
    lib.rpca_status_str.restype = ctypes.c_char_p
    lib.rpca_set_device_panel_cb.argtypes = [vp, DEVICE_PANEL_CB, vp]
    lib.rpca_set_device_panel_cb.restype = i32
    lib.rpca_destroy.argtypes = [vp]
    lib.rpca_destroy.restype = None
    _lib = lib
    return lib


class RPCAError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        name = STATUS_NAMES.get(code, str(code))
        msg = load().rpca_status_str(code).decode()
        super().__init__(f"{where}: {name} ({msg})")


def check(code: int, where: str):
    if code != RPCA_OK:
        raise RPCAError(code, where)
