"""Counter-based random streams for the seeded synthetic inputs.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from its published definition: a 4x32-bit
counter and a 2x32-bit key go through ten rounds; each round multiplies
words 0 and 2 by two fixed odd constants, mixes the high halves with the
other words and the key, and the key is bumped by two Weyl constants between
rounds.

Element addressing (shared with the GPU twin in ``synth/csrc``): element ``e``
(64-bit) of stream ``s`` under seed ``seed`` uses the block

    counter = (b & 0xffffffff, b >> 32, s, 0),   b = e >> 1
    key     = (seed & 0xffffffff, seed >> 32)

and takes half ``e & 1`` of the block's output.  A block's four words give two
53-bit uniforms u1 = (x0,x1), u2 = (x2,x3), each (k + 1/2) * 2^-53 so they lie
strictly inside (0, 1).  Normals use Box-Muller in float64:
z0 = sqrt(-2 ln u1) cos(2 pi u2) (half 0), z1 = ... sin(2 pi u2) (half 1).
Uniform streams return u1 for half 0 and u2 for half 1.

This module holds no arithmetic of the PCA method itself; it only produces the
random inputs that both the oracle and the GPU path consume.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)
_TWO_M53 = 2.0 ** -53


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten-round Philox4x32 on arrays of 32-bit words; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32).copy()
    c1 = np.asarray(c1, dtype=np.uint32).copy()
    c2 = np.asarray(c2, dtype=np.uint32).copy()
    c3 = np.asarray(c3, dtype=np.uint32).copy()
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = np.uint32((int(k0) + int(W0)) & 0xFFFFFFFF)
                k1 = np.uint32((int(k1) + int(W1)) & 0xFFFFFFFF)
            p0 = c0.astype(np.uint64) * M0
            p1 = c2.astype(np.uint64) * M1
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _blocks(seed: int, stream: int, start: int, count: int):
    e = np.arange(start, start + count, dtype=np.uint64)
    b = e >> np.uint64(1)
    half = (e & np.uint64(1)).astype(bool)
    b_lo = (b & _MASK32).astype(np.uint32)
    b_hi = (b >> np.uint64(32)).astype(np.uint32)
    s = np.full(e.shape, stream & 0xFFFFFFFF, dtype=np.uint32)
    z = np.zeros(e.shape, dtype=np.uint32)
    x0, x1, x2, x3 = philox4x32_10(b_lo, b_hi, s, z, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return half, x0, x1, x2, x3


def _u53(hi32, lo32):
    k = (hi32.astype(np.uint64) >> np.uint64(5)) * np.uint64(1 << 26) + (lo32.astype(np.uint64) >> np.uint64(6))
    return (k.astype(np.float64) + 0.5) * _TWO_M53


def normals(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Standard normal float64 values for elements [start, start+count) of a stream."""
    if count <= 0:
        return np.zeros(0, dtype=np.float64)
    half, x0, x1, x2, x3 = _blocks(seed, stream, start, count)
    u1 = _u53(x0, x1)
    u2 = _u53(x2, x3)
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return np.where(half, r * np.sin(t), r * np.cos(t))


def uniforms(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Uniform(0,1) float64 values for elements [start, start+count) of a stream."""
    if count <= 0:
        return np.zeros(0, dtype=np.float64)
    half, x0, x1, x2, x3 = _blocks(seed, stream, start, count)
    return np.where(half, _u53(x2, x3), _u53(x0, x1))


def normal_matrix(seed: int, stream: int, rows: int, cols: int, row0: int = 0,
                  chunk_rows: int | None = None) -> np.ndarray:
    """Rows [row0, row0+rows) of a row-major Gaussian matrix with ``cols`` columns.

    Element (r, c) is stream element r*cols + c, so any row panel can be
    regenerated on its own.
    """
    out = np.empty((rows, cols), dtype=np.float64)
    step = chunk_rows or max(1, (1 << 22) // max(cols, 1))
    for r in range(0, rows, step):
        rr = min(step, rows - r)
        out[r:r + rr] = normals(seed, stream, (row0 + r) * cols, rr * cols).reshape(rr, cols)
    return out
