"""Reference definitions of the stored formats of A (test infrastructure).

These are the plain definitions the quantised storage must follow, written
with NumPy only; the GPU quantiser is checked against them bit for bit, and
the oracle factorises the dequantised values they define.

* bfloat16: the upper 16 bits of a float32 after round-to-nearest-even.
* hi + lo:  hi = bf16(a), lo = bf16(a - hi) (a - hi is exact in float32).
* FP8 E4M3 (OCP 8-bit floating point, "E4M3"): 1 sign bit, 4 exponent bits
  with bias 7, 3 mantissa bits, subnormals, no infinities, the all-ones
  pattern S.1111.111 is NaN, largest finite magnitude 448.  Values are
  rounded to nearest, ties to even, and saturated at +-448.  Each column j
  carries a float32 scale c_j = max_i |a_ij| / 448 (1 for a zero column) and
  the stored code is e4m3(a_ij / c_j) with the division done in float32.
"""
from __future__ import annotations

import numpy as np


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even); returns uint16 bit patterns."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    return (rounded & np.uint64(0xFFFF)).astype(np.uint16)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def hilo_bits(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_bits(x)
    lo = bf16_bits((x - bf16_to_f32(hi)).astype(np.float32))
    return hi, lo


def _e4m3_table() -> np.ndarray:
    """Value of every e4m3 code 0..255 (NaN for S.1111.111)."""
    v = np.empty(256, dtype=np.float64)
    for q in range(256):
        s = -1.0 if q & 0x80 else 1.0
        e = (q >> 3) & 0xF
        mt = q & 7
        if e == 0xF and mt == 7:
            v[q] = np.nan
        elif e == 0:
            v[q] = s * mt / 8.0 * 2.0 ** -6
        else:
            v[q] = s * (1.0 + mt / 8.0) * 2.0 ** (e - 7)
    return v


E4M3 = _e4m3_table()


def e4m3_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to e4m3 codes: nearest, ties to the even code, saturating at 448."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    pos = E4M3[:0x7F]                      # codes 0..126: 0 .. 448, increasing
    a = np.minimum(np.abs(x), 448.0)
    idx = np.searchsorted(pos, a)          # first code with value >= a
    idx = np.clip(idx, 1, 0x7E)
    lo, hi = pos[idx - 1], pos[idx]
    take_hi = (a - lo > hi - a) | ((a - lo == hi - a) & ((idx & 1) == 0))
    code = np.where(take_hi, idx, idx - 1)
    code = np.where(a >= 448.0, 0x7E, code)
    code = np.where(a == 0.0, 0, code)
    sign = np.where((x < 0) & (code != 0), 0x80, 0)
    return (code | sign).astype(np.uint8)


def fp8_quantize(A: np.ndarray):
    """Per-column scales and e4m3 codes of a float32 matrix."""
    A = np.asarray(A, dtype=np.float32)
    amax = np.abs(A).max(axis=0)
    scale = np.where(amax > 0, (amax / np.float32(448.0)).astype(np.float32), np.float32(1.0)).astype(np.float32)
    q = e4m3_bits((A / scale[None, :]).astype(np.float32))
    return q, scale


def fp8_dequantize(q: np.ndarray, scale: np.ndarray) -> np.ndarray:
    return E4M3[np.asarray(q, dtype=np.uint8)] * np.asarray(scale, dtype=np.float64)[None, :]


def dequantize(storage: str, data, scale=None) -> np.ndarray:
    """float64 values of a stored matrix: 'bf16' -> bits, 'bf16_hilo' -> (hi, lo), 'fp8_e4m3' -> codes + scale."""
    if storage == "f32":
        return np.asarray(data, dtype=np.float64)
    if storage == "bf16":
        return bf16_to_f32(data).astype(np.float64)
    if storage == "bf16_hilo":
        hi, lo = data
        return bf16_to_f32(hi).astype(np.float64) + bf16_to_f32(lo).astype(np.float64)
    if storage == "fp8_e4m3":
        return fp8_dequantize(data, scale)
    raise ValueError(storage)


def quantize(storage: str, A: np.ndarray, shift: np.ndarray | None = None):
    """Stored representation of float32 A (optionally of A - 1 shift^T, subtracted in float32).

    Returns (data, scale): bf16 -> uint16 bits; bf16_hilo -> (hi, lo); fp8_e4m3 -> (codes, scale).
    """
    A = np.asarray(A, dtype=np.float32)
    if shift is not None:
        A = (A - np.asarray(shift, dtype=np.float32)[None, :]).astype(np.float32)
    if storage == "bf16":
        return bf16_bits(A), None
    if storage == "bf16_hilo":
        return hilo_bits(A), None
    if storage == "fp8_e4m3":
        q, s = fp8_quantize(A)
        return q, s
    raise ValueError(storage)
