"""Device-side twin of the seeded generator, for inputs too large to build on the host.

``build()`` compiles ``synth/csrc/synth_kernels.hip`` into ``synth/libsynth.so``.
The functions take torch tensors for device memory and mirror
``synth.fixtures.lowrank_noise_panel`` and ``synth.philox.normals``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "synth_kernels.hip")
LIB = os.path.join(HERE, "libsynth.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
_lib = None


def build() -> str:
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", SRC, "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("synth build failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} missing; run synth.gpu.build()")
        lib = ctypes.CDLL(LIB)
        vp, i64, i32, u64, u32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_double)
        lib.synth_lowrank_noise.argtypes = [vp, i64, i64, i64, i64, vp, i32, vp, vp, dbl, vp, u64, u32, vp]
        lib.synth_lowrank_noise.restype = i32
        lib.synth_normals.argtypes = [vp, u64, u32, u64, i64, vp]
        lib.synth_normals.restype = i32
        _lib = lib
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def lowrank_noise_into(A, row0, Ur, sigma, Vr, noise, offsets, seed, noise_stream=4):
    """Fill the device float32 tensor A (rows x n view, row-major) with rows [row0, row0+rows)."""
    rows, n = A.shape
    rc = load().synth_lowrank_noise(
        ctypes.c_void_p(A.data_ptr()), A.stride(0), rows, n, row0, ctypes.c_void_p(Ur.data_ptr()), Ur.shape[1],
        ctypes.c_void_p(sigma.data_ptr()), ctypes.c_void_p(Vr.data_ptr()), float(noise),
        ctypes.c_void_p(offsets.data_ptr()) if offsets is not None else ctypes.c_void_p(0), int(seed),
        int(noise_stream), _stream())
    if rc != 0:
        raise RuntimeError(f"synth_lowrank_noise failed ({rc})")


def normals(out, seed, stream_id, start):
    rc = load().synth_normals(ctypes.c_void_p(out.data_ptr()), int(seed), int(stream_id), int(start), out.numel(),
                              _stream())
    if rc != 0:
        raise RuntimeError(f"synth_normals failed ({rc})")
