"""Device-side twin of the seeded generator, for inputs too large to build on the host.

``build()`` compiles ``synth/csrc/synth_kernels.hip`` into ``synth/libsynth.so``.
The functions take torch tensors for device memory and mirror
``synth.fixtures.lowrank_noise_panel`` and ``synth.philox.normals``.
"""
from __future__ import annotations

import ctypes
import math
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
        lib.synth_copy_rows.argtypes = [vp, i64, vp, i64, i64, i64, vp]
        lib.synth_copy_rows.restype = i32
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


def lowrank_noise_at(dst, ld, rows, n, row0, Ur, sigma, Vr, noise, offsets, seed, stream, noise_stream=4):
    """As lowrank_noise_into, for a raw device address `dst` (leading dimension ld) on HIP stream `stream`."""
    rc = load().synth_lowrank_noise(
        ctypes.c_void_p(dst), ld, rows, n, row0, ctypes.c_void_p(Ur.data_ptr()), Ur.shape[1],
        ctypes.c_void_p(sigma.data_ptr()), ctypes.c_void_p(Vr.data_ptr()), float(noise),
        ctypes.c_void_p(offsets.data_ptr()) if offsets is not None else ctypes.c_void_p(0), int(seed),
        int(noise_stream), ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"synth_lowrank_noise failed ({rc})")


def copy_rows_at(dst, ld, src, row0, rows, stream):
    """Rows [row0, row0+rows) of the device float32 tensor src into the raw device address dst (ld) on `stream`."""
    n = src.shape[1]
    rc = load().synth_copy_rows(ctypes.c_void_p(dst), ld, ctypes.c_void_p(src[row0:row0 + rows].data_ptr()),
                                src.stride(0), rows, n, ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"synth_copy_rows failed ({rc})")


def normals(out, seed, stream_id, start):
    rc = load().synth_normals(ctypes.c_void_p(out.data_ptr()), int(seed), int(stream_id), int(start), out.numel(),
                              _stream())
    if rc != 0:
        raise RuntimeError(f"synth_normals failed ({rc})")


def example_dct_rows(which: int, m: int, n: int, out, chunk_bytes: int = 1 << 32):
    """Fill ``out`` (an m x n float32 tensor, any device) with A = E S F of the paper's first or second
    example (Section 6.1): E, F unitary DCT-II of orders m and n (first n columns of E), S the
    example's diagonal.  Matches ``synth.fixtures.example_dct(which, m, n)["A"]``.

    A row of A is the inverse DCT (DCT-III) of sigma o E[r, :n], done in float64 as one complex FFT of
    length 2n per row, so the cost is O(m n log n) rather than the O(m n^2) of forming E S F.
    """
    import torch
    from .fixtures import example1_sigma, example2_sigma

    if m < n:
        raise ValueError("the examples have m >= n")
    dev = out.device
    sigma = example1_sigma(n) if which == 1 else example2_sigma(n)
    j = torch.arange(n, dtype=torch.float64, device=dev)
    # F[j][c] = sqrt(2/n) a_j cos(pi (2c+1) j / (2n)): row r of A is Re(sum_j w_j x_j e^{2 pi i j c / (2n)})
    # with x = sigma o E[r, :] and w_j = sqrt(2/n) a_j e^{i pi j / (2n)}
    w = torch.polar(torch.full((n,), math.sqrt(2.0 / n), dtype=torch.float64, device=dev), math.pi * j / (2.0 * n))
    w[0] = w[0] / math.sqrt(2.0)
    w = w * torch.from_numpy(sigma).to(dev)
    twoj1 = 2.0 * j + 1.0
    rows = max(1, min(m, chunk_bytes // (16 * 2 * n * 3)))
    for r0 in range(0, m, rows):
        r1 = min(m, r0 + rows)
        r = torch.arange(r0, r1, dtype=torch.float64, device=dev)
        # E[r][j] = sqrt(2/m) a_r cos(pi (2j+1) r / (2m)); (2j+1) r mod 4m is exact in float64
        ph = torch.remainder(torch.outer(r, twoj1), 4.0 * m)
        E = torch.cos(ph * (math.pi / (2.0 * m))) * math.sqrt(2.0 / m)
        if r0 == 0:
            E[0] /= math.sqrt(2.0)
        Z = torch.fft.ifft(E * w, n=2 * n, dim=1)
        out[r0:r1] = (Z[:, :n].real * (2.0 * n)).to(out.dtype)
        del E, Z, ph
    return sigma
