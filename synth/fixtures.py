"""Seeded synthetic problems with known spectra (inputs only, no PCA arithmetic).

Every matrix is addressable by row panel: a panel [row0, row0+rows) can be
rebuilt without the rest, which is what the out-of-core and callback sources
need.  Factor matrices are float64; the stored data matrix A is float32 with
round-to-nearest-even from the float64 value, the storage precision the paper
uses for the matrix on disk (Section 6, opening paragraphs).

Workloads
---------
* ``svd_problem``: A = U diag(sigma) V^T with Haar U, V (QR of a Gaussian,
  diag(R) > 0).  With sigma_j = 0.9^(j-1), m=2000, n=1000 this is the small
  plain-method case; with sigma_j = 2*0.95^(j-1) it is the differentiation case.
* ``lowrank_noise_panel``: A = U_r diag(sigma) V_r^T + noise*N + 1 c^T with
  orthonormalised Gaussian U_r, V_r, iid N(0,1) noise N and column offsets
  c_j ~ U(0,1) (c = 0 when no offsets are asked for).  This is the in-core
  (200000 x 20000, r=50, sigma_j=1/j, noise 1e-3, offsets) and the streaming
  (r=100, sigma_j=exp(-j/20), noise 1e-4, no offsets) structure.
* ``example_dct``: A = E S F with unitary DCT-II matrices E, F and the paper's
  diagonal S of its first and second examples (Section 6.1).
"""
from __future__ import annotations

import math
import numpy as np

from .philox import normals, uniforms, normal_matrix

# stream ids inside one seed
STREAM_G = 1
STREAM_U = 2
STREAM_V = 3
STREAM_NOISE = 4
STREAM_SHIFT = 5
STREAM_W = 6
STREAM_GU = 7
STREAM_GV = 8
STREAM_EST = 9
STREAM_DIR = 10


def to_f32(x: np.ndarray) -> np.ndarray:
    """Round float64 to float32 (numpy's cast is round-to-nearest-even)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def gaussian_G(seed: int, n: int, l: int, stream: int = STREAM_G) -> np.ndarray:
    """The n x l Gaussian test matrix as float32, element (r, c) = stream element r*l + c."""
    return to_f32(normal_matrix(seed, stream, n, l))


def orthonormal_columns(Z: np.ndarray) -> np.ndarray:
    """Q factor of Z with the sign fixed so that diag(R) > 0 (Haar when Z is Gaussian)."""
    Q, R = np.linalg.qr(Z, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def haar(seed: int, stream: int, rows: int, cols: int) -> np.ndarray:
    return orthonormal_columns(normal_matrix(seed, stream, rows, cols))


def svd_problem(seed: int, m: int, n: int, sigma: np.ndarray):
    """A = U diag(sigma) V^T (float64 factors) and its float32 storage."""
    r = len(sigma)
    U = haar(seed, STREAM_U, m, r)
    V = haar(seed, STREAM_V, n, r)
    A64 = (U * sigma) @ V.T
    return {"A": to_f32(A64), "A64": A64, "U": U, "V": V, "sigma": np.asarray(sigma, dtype=np.float64)}


def plain_small(seed: int = 1007, m: int = 2000, n: int = 1000):
    """Small plain-method case: sigma_j = 0.9^(j-1), j <= n; k=10, l=12, i=1."""
    sigma = 0.9 ** np.arange(min(m, n), dtype=np.float64)
    p = svd_problem(seed, m, n, sigma)
    p.update(k=10, l=12, i=1, center=False, G=gaussian_G(seed, n, 12))
    return p


def diff_problem(seed: int = 5510, m: int = 2000, n: int = 800, k: int = 16, l: int = 24, i: int = 2):
    """Differentiation case: sigma_j = 2*0.95^(j-1) with distinct gaps."""
    sigma = 2.0 * 0.95 ** np.arange(min(m, n), dtype=np.float64)
    p = svd_problem(seed, m, n, sigma)
    p.update(k=k, l=l, i=i, center=False, G=gaussian_G(seed, n, l))
    return p


def lowrank_factors(seed: int, m: int, n: int, r: int):
    """Orthonormalised Gaussian U_r (m x r) and V_r (n x r)."""
    return haar(seed, STREAM_U, m, r), haar(seed, STREAM_V, n, r)


def column_offsets(seed: int, n: int) -> np.ndarray:
    return uniforms(seed, STREAM_SHIFT, 0, n)


def lowrank_noise_panel(seed: int, Ur: np.ndarray, sigma: np.ndarray, Vr: np.ndarray,
                        noise: float, offsets: np.ndarray | None, row0: int, rows: int,
                        as_f64: bool = False) -> np.ndarray:
    """Rows [row0, row0+rows) of U_r diag(sigma) V_r^T + noise*N + 1 c^T.

    The low-rank term is summed in float64 in the order j = 0..r-1, then the
    noise and the offset are added and the float64 value is rounded once to
    float32.
    """
    n = Vr.shape[0]
    Ub = Ur[row0:row0 + rows] * sigma
    acc = np.zeros((rows, n), dtype=np.float64)
    for j in range(Ur.shape[1]):
        acc += np.outer(Ub[:, j], Vr[:, j])
    acc += noise * normal_matrix(seed, STREAM_NOISE, rows, n, row0=row0)
    if offsets is not None:
        acc += offsets[None, :]
    return acc if as_f64 else to_f32(acc)


def lowrank_noise(seed: int, m: int, n: int, r: int, sigma: np.ndarray, noise: float,
                  with_offsets: bool, panel_rows: int = 4096):
    Ur, Vr = lowrank_factors(seed, m, n, r)
    c = column_offsets(seed, n) if with_offsets else None
    A = np.empty((m, n), dtype=np.float32)
    for r0 in range(0, m, panel_rows):
        rr = min(panel_rows, m - r0)
        A[r0:r0 + rr] = lowrank_noise_panel(seed, Ur, sigma, Vr, noise, c, r0, rr)
    return {"A": A, "Ur": Ur, "Vr": Vr, "sigma": sigma, "offsets": c, "noise": noise}


def incore_problem(seed: int = 2020, m: int = 200000, n: int = 20000, r: int = 50,
                   k: int = 50, l: int = 60, i: int = 2):
    """Low-rank + 1e-3 noise + U(0,1) column offsets; sigma_j = 1/j; centred factorisation."""
    sigma = 1.0 / np.arange(1, r + 1, dtype=np.float64)
    p = lowrank_noise(seed, m, n, r, sigma, 1e-3, True)
    p.update(k=k, l=l, i=i, center=True, G=gaussian_G(seed, n, l))
    return p


def stream_problem(seed: int = 4000, m: int = 4_000_000, n: int = 25_000, r: int = 100,
                   k: int = 100, l: int = 120, i: int = 2):
    """Streaming structure: rank 100, sigma_j = exp(-j/20), noise 1e-4, no offsets."""
    sigma = np.exp(-np.arange(1, r + 1, dtype=np.float64) / 20.0)
    p = lowrank_noise(seed, m, n, r, sigma, 1e-4, False)
    p.update(k=k, l=l, i=i, center=False, G=gaussian_G(seed, n, l))
    return p


def dct2_matrix(N: int) -> np.ndarray:
    """Unitary DCT-II matrix C with C[f, t] = sqrt(2/N) a_f cos(pi (2t+1) f / (2N)), a_0 = 1/sqrt(2)."""
    f = np.arange(N, dtype=np.float64)[:, None]
    t = np.arange(N, dtype=np.float64)[None, :]
    C = math.sqrt(2.0 / N) * np.cos(np.pi * (2.0 * t + 1.0) * f / (2.0 * N))
    C[0] *= 1.0 / math.sqrt(2.0)
    return C


def example1_sigma(n: int) -> np.ndarray:
    """Diagonal of S in the first example: 10^(-4(j-1)/19) for j <= 20, 10^-4/(j-20)^(1/10) after."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.where(j <= 20, 10.0 ** (-4.0 * (j - 1.0) / 19.0), 1e-4 / np.maximum(j - 20.0, 1.0) ** 0.1)


def example2_sigma(n: int) -> np.ndarray:
    """Diagonal of S in the second example: plateaus 1, .67, .34, .01, then a linear ramp to 0."""
    j = np.arange(1, n + 1, dtype=np.float64)
    s = np.empty(n, dtype=np.float64)
    s[j <= 3] = 1.00
    s[(j >= 4) & (j <= 6)] = 0.67
    s[(j >= 7) & (j <= 9)] = 0.34
    s[(j >= 10) & (j <= 12)] = 0.01
    tail = j >= 13
    s[tail] = 0.01 * (n - j[tail]) / (n - 13.0)
    return s


def example_dct(which: int, m: int, n: int):
    """A = E S F with E, F unitary DCT-II of orders m, n (the paper's first two examples)."""
    sigma = example1_sigma(n) if which == 1 else example2_sigma(n)
    E = dct2_matrix(m)
    F = dct2_matrix(n)
    A64 = (E[:, :n] * sigma) @ F
    return {"A": to_f32(A64), "A64": A64, "sigma": sigma, "U": E[:, :n], "V": F.T}


def backward_weights(seed: int, m: int, n: int, k: int):
    """Loss weights w, G_U, G_V of the differentiation case (iid N(0,1))."""
    w = normals(seed, STREAM_W, 0, k)
    GU = normal_matrix(seed, STREAM_GU, m, k)
    GV = normal_matrix(seed, STREAM_GV, n, k)
    return w, GU, GV
