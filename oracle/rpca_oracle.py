"""Float64 CPU oracle of the randomized block-Lanczos PCA (Halko, Martinsson,
Shkolnisky, Tygert, "An algorithm for the principal component analysis of
large data sets").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module;
only the tests, the smoke entry point and the benchmark's CPU-baseline leg may
call it.  It shares no code with the GPU library: the only thing both sides
use is the seeded input generator in ``synth``.

What it computes
----------------
Section 3 ("Summary of the algorithm"), Steps 1-6, in the paper's order and
notation, with the stored matrix A (float32 values) upcast exactly to float64
and processed one row panel at a time the way Section 4.2 ("Computations with
storage on disk") describes:

* Step 1: H^(0) = A G (eq. first_prod); H^(j) = A (A^T H^(j-1)) for j = 1..i
  (eqs. second_prod .. last_prod), each A^T H^(j-1) formed first as F and then
  A F, as Section 4.2 does; H = [H^(0) | ... | H^(i)] (eq. product23).
* Step 2: pivoted QR, H = Q R (eq. good_approx23), via LAPACK dgeqp3.
* Step 3: T = A^T Q (eq. product_t3), by accumulating the transposes of the
  rows of A weighted by the rows of Q.
* Step 4: T = V~ S~ W^T (eq. svd_small3), S~ non-increasing, via LAPACK dgesdd.
* Step 5: U~ = Q W (eq. product33).
* Step 6: U, S, V = leftmost k columns / leading k x k block.

Centering (Introduction: normalise A by subtracting from each column its
mean) is applied by materialising each panel of A - 1 mu^T in float64, with
mu the exact float64 column mean of the stored A.

Readings where the paper is silent (each is also listed in the design notes):
* parameters: l >= k, (i+1) l <= n - k and k < min(m, n) (Section 3);
* sign of each singular pair: (u_j, v_j) is flipped so the entry of v_j with
  the largest magnitude is positive, ties going to the lowest index;
* a rank-deficient H keeps all (i+1) l columns of Q (LAPACK's economic QR).

The Appendix spectral-norm estimator p_{j,k}(D) and the bound of eq.
sort_of_svd are provided for the accuracy checks.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.linalg

PANEL_ROWS = 16384


class PanelReader:
    """Row-panel access to a row-major matrix (Section 4.2), counting entries read."""

    def __init__(self, A, panel_rows: int = PANEL_ROWS, center_mean: np.ndarray | None = None):
        self.A = A
        self.m, self.n = A.shape
        self.panel_rows = max(1, int(panel_rows))
        self.mu = center_mean
        self.entries_read = 0

    def panels(self):
        for r0 in range(0, self.m, self.panel_rows):
            r1 = min(self.m, r0 + self.panel_rows)
            P = np.asarray(self.A[r0:r1], dtype=np.float64)
            self.entries_read += P.size
            if self.mu is not None:
                P = P - self.mu[None, :]
            yield r0, r1, P


def column_mean(A, panel_rows: int = PANEL_ROWS) -> np.ndarray:
    """Exact float64 column means of the stored A, one panel at a time."""
    m, n = A.shape
    s = np.zeros(n, dtype=np.float64)
    for r0 in range(0, m, panel_rows):
        s += np.asarray(A[r0:r0 + panel_rows], dtype=np.float64).sum(axis=0)
    return s / m


def apply_A(reader: PanelReader, X: np.ndarray) -> np.ndarray:
    """A X formed panel by panel: each block of rows of A times X (Section 4.2)."""
    out = np.empty((reader.m, X.shape[1]), dtype=np.float64)
    for r0, r1, P in reader.panels():
        out[r0:r1] = P @ X
    return out


def apply_At(reader: PanelReader, Y: np.ndarray) -> np.ndarray:
    """A^T Y: start from zeros and add the transposes of the rows of A weighted by Y (Section 4.2)."""
    out = np.zeros((reader.n, Y.shape[1]), dtype=np.float64)
    for r0, r1, P in reader.panels():
        out += P.T @ Y[r0:r1]
    return out


def check_params(m: int, n: int, k: int, l: int, i: int) -> None:
    """Section 3 preconditions: k < min(m, n), l >= k, (i+1) l <= n - k (with n <= m)."""
    small = min(m, n)
    if not (1 <= k < small):
        raise ValueError(f"need 1 <= k < min(m, n); got k={k}, m={m}, n={n}")
    if l < k:
        raise ValueError(f"need l >= k; got l={l}, k={k}")
    if i < 0:
        raise ValueError("need i >= 0")
    if (i + 1) * l > small - k:
        raise ValueError(f"need (i+1) l <= min(m,n) - k; got (i+1)l={(i + 1) * l}, bound={small - k}")


def sign_convention(Vt: np.ndarray):
    """+1/-1 per column so that the largest-magnitude entry of each column is positive (first on ties)."""
    idx = np.argmax(np.abs(Vt), axis=0)
    s = np.sign(Vt[idx, np.arange(Vt.shape[1])])
    s[s == 0] = 1.0
    return s


@dataclass
class RPCAResult:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    mu: np.ndarray | None = None
    H_blocks: list = field(default_factory=list)
    F_blocks: list = field(default_factory=list)
    Q: np.ndarray | None = None
    R: np.ndarray | None = None
    piv: np.ndarray | None = None
    T: np.ndarray | None = None
    Vtilde: np.ndarray | None = None
    Stilde: np.ndarray | None = None
    W: np.ndarray | None = None
    entries_read: int = 0


def rpca(A, k: int, l: int, i: int, G: np.ndarray, center: bool = False,
         panel_rows: int = PANEL_ROWS, validate: bool = True) -> RPCAResult:
    """Steps 1-6 of Section 3 on the stored A (m x n, m >= n) with the given n x l test matrix G."""
    m, n = A.shape
    if n > m:
        # Section 3 assumes n <= m and applies the algorithm to A^T otherwise.
        Ac = np.asarray(A, dtype=np.float64)
        if center:
            Ac = Ac - Ac.mean(axis=0)[None, :]
        r = rpca(Ac.T, k, l, i, G, center=False, panel_rows=panel_rows, validate=validate)
        r.U, r.V = r.V, r.U
        return r
    if validate:
        check_params(m, n, k, l, i)
    G = np.asarray(G, dtype=np.float64)
    if G.shape != (n, l):
        raise ValueError(f"G must be {n} x {l}")
    mu = column_mean(A, panel_rows) if center else None
    reader = PanelReader(A, panel_rows, mu)

    # Step 1: H^(0) = A G; H^(j) = A (A^T H^(j-1)), with F = A^T H^(j-1) formed first.
    H_blocks = [apply_A(reader, G)]
    F_blocks = []
    for _ in range(i):
        F = apply_At(reader, H_blocks[-1])
        F_blocks.append(F)
        H_blocks.append(apply_A(reader, F))
    r = steps_2_to_6(reader, H_blocks, k)
    r.mu, r.F_blocks = mu, F_blocks
    return r


def steps_2_to_6(reader: PanelReader, H_blocks: list, k: int) -> RPCAResult:
    """Steps 2-6 of Section 3 from the blocks H^(0..i) of Step 1, reading A through ``reader``."""
    H = np.hstack(H_blocks)

    # Step 2: pivoted QR of H; Q has (i+1) l orthonormal columns.
    Q, R, piv = scipy.linalg.qr(H, mode="economic", pivoting=True)

    # Step 3: T = A^T Q.
    T = apply_At(reader, Q)

    # Step 4: SVD of T, singular values non-increasing.
    Vt, St, WT = np.linalg.svd(T, full_matrices=False)
    W = WT.T

    # sign of each singular pair (reading: largest-magnitude entry of v_j positive)
    s = sign_convention(Vt)
    Vt = Vt * s
    W = W * s

    # Step 5: U~ = Q W.
    Ut = Q @ W

    # Step 6: leftmost k columns and the leading k x k block.
    return RPCAResult(U=Ut[:, :k].copy(), S=St[:k].copy(), V=Vt[:, :k].copy(),
                      H_blocks=H_blocks, Q=Q, R=R, piv=piv, T=T,
                      Vtilde=Vt, Stilde=St, W=W, entries_read=reader.entries_read)


def error_bound(k: int, n: int, i: int, sigma_k1: float, C: float = 100.0) -> float:
    """Right-hand side of eq. sort_of_svd: sqrt((C k n)^(1/(2i+1)) + min(1, C/n)) * sigma_{k+1}."""
    return math.sqrt((C * k * n) ** (1.0 / (2 * i + 1)) + min(1.0, C / n)) * sigma_k1


def _centered_dense(A, center: bool) -> np.ndarray:
    A64 = np.asarray(A, dtype=np.float64)
    if center:
        A64 = A64 - A64.mean(axis=0)[None, :]
    return A64


def residual_exact(A, U, S, V, center: bool = False) -> float:
    """||A~ - U S V^T||_2 by a dense SVD of the difference (small inputs)."""
    D = _centered_dense(A, center) - (np.asarray(U, np.float64) * np.asarray(S, np.float64)) @ np.asarray(V, np.float64).T
    return float(np.linalg.norm(D, 2))


def residual_gram(A, U, S, V, center: bool = False, panel_rows: int = PANEL_ROWS) -> float:
    """||D||_2 with D = A~ - U S V^T from the n x n Gram D^T D (exact for any U, S, V).

    D^T D = A~^T A~ - A~^T U S V^T - V S U^T A~ + V S (U^T U) S V^T, formed with
    one panel pass for A~^T A~ and A~^T U.
    """
    m, n = A.shape
    mu = column_mean(A, panel_rows) if center else None
    U = np.asarray(U, np.float64)
    S = np.asarray(S, np.float64)
    V = np.asarray(V, np.float64)
    GA = np.zeros((n, n))
    AU = np.zeros((n, U.shape[1]))
    for r0 in range(0, m, panel_rows):
        P = np.asarray(A[r0:r0 + panel_rows], dtype=np.float64)
        if mu is not None:
            P = P - mu[None, :]
        GA += P.T @ P
        AU += P.T @ U[r0:r0 + panel_rows]
    VS = V * S
    M = GA - AU @ VS.T - VS @ AU.T + VS @ (U.T @ U) @ VS.T
    M = 0.5 * (M + M.T)
    lam = scipy.linalg.eigh(M, eigvals_only=True, subset_by_index=[n - 1, n - 1])[0]
    return float(math.sqrt(max(lam, 0.0)))


def estimate_norm(apply_D, apply_Dt, starts: np.ndarray, j: int = 6) -> float:
    """Appendix estimator p_{j,k}(D) = max_q sqrt(||(D^T D)^j w_q|| / ||(D^T D)^(j-1) w_q||).

    ``starts`` holds the k start vectors w_q (n x k) with iid N(0,1) entries.
    Each iterate is divided by its norm before the next product; this changes
    neither the ratio nor the maximum, it only keeps the powers in range.
    """
    best = 0.0
    for q in range(starts.shape[1]):
        x = np.asarray(starts[:, q], dtype=np.float64)
        x = x / np.linalg.norm(x)
        ratio = 0.0
        for _ in range(j):
            y = apply_Dt(apply_D(x))
            ratio = np.linalg.norm(y) / np.linalg.norm(x)
            nrm = np.linalg.norm(y)
            if nrm == 0.0:
                break
            x = y / nrm
        best = max(best, math.sqrt(ratio))
    return best


def residual_estimate(A, U, S, V, starts: np.ndarray, center: bool = False, j: int = 6,
                      panel_rows: int = PANEL_ROWS) -> float:
    """p_{j,k}(A~ - U S V^T) with the Appendix's j = 6 by default, applying D and D^T by panels."""
    mu = column_mean(A, panel_rows) if center else None
    reader = PanelReader(A, panel_rows, mu)
    U = np.asarray(U, np.float64)
    S = np.asarray(S, np.float64)
    V = np.asarray(V, np.float64)

    def D(x):
        return apply_A(reader, x[:, None])[:, 0] - U @ (S * (V.T @ x))

    def Dt(y):
        return apply_At(reader, y[:, None])[:, 0] - V @ (S * (U.T @ y))

    return estimate_norm(D, Dt, starts, j)


def estimator_failure_bound(n: int, j: int, k: int) -> float:
    """Appendix eq. high_prob: P[p_{j,k}(D) < ||D||/2] < (2n / ((2j-1) 16^j))^(k/2)."""
    return (2.0 * n / ((2 * j - 1) * 16.0 ** j)) ** (k / 2.0)
