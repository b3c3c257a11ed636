"""Reverse-mode derivative of the randomized PCA (test infrastructure, CPU, float64).

The paper defines no derivative.  The quantity computed here is the exact
derivative of Steps 1-6 of Section 3 as a function of A, with the Gaussian
test matrix G held fixed (the randomness is an input):

    A~ = A - 1 mu^T (centring) or A;  H^(0) = A~ G, H^(j) = A~ (A~^T H^(j-1));
    H = [H^(0) .. H^(i)] = Q R;  T = A~^T Q = V~ S~ W^T;
    U = Q W[:, :k], S = S~[:k], V = V~[:, :k], columns signed so that the
    largest-magnitude entry of each v_j is positive.

It is written with torch (CPU, float64) and differentiated by autograd; QR
and SVD enter as library steps.  The positive per-block rescaling of the
power iterates that the GPU uses against overflow (Section 3, remark on
floating-point range) leaves span(H), hence Q and every output, unchanged,
so it is absent here.  The pinning tests check this function against
central finite differences of its own forward and against closed forms
(the derivative of a singular value, u_j v_j^T, when the range is captured
exactly), independently of any GPU code.
"""
from __future__ import annotations

import numpy as np
import torch


def forward(A: torch.Tensor, k: int, l: int, i: int, G: torch.Tensor, center: bool = False):
    """Steps 1-6 of Section 3 on a float64 torch matrix (m >= n); returns (U, S, V)."""
    Ac = A - A.mean(dim=0, keepdim=True) if center else A
    X = G
    blocks = []
    for j in range(i + 1):
        Hj = Ac @ X                      # first_prod / later products of Step 1
        blocks.append(Hj)
        if j < i:
            X = Ac.T @ Hj
    H = torch.cat(blocks, dim=1)
    Q, _ = torch.linalg.qr(H)            # Step 2 (span(H); pivoting does not change it)
    T = Ac.T @ Q                         # Step 3
    Vt, St, Wh = torch.linalg.svd(T, full_matrices=False)   # Step 4: T = V~ S~ W^T
    W = Wh.T
    U = Q @ W[:, :k]                     # Step 5
    V = Vt[:, :k]
    S = St[:k]
    with torch.no_grad():                # sign convention: largest |v_ij| positive (piecewise constant)
        idx = torch.argmax(V.abs(), dim=0)
        sgn = torch.sign(V[idx, torch.arange(k)])
        sgn[sgn == 0] = 1.0
    return U * sgn, S, V * sgn


def loss_value(U, S, V, gS, gU, gV) -> torch.Tensor:
    """<gS, S> + <gU, U> + <gV, V> (any cotangent may be None)."""
    val = torch.zeros((), dtype=torch.float64)
    if gS is not None:
        val = val + (S * gS).sum()
    if gU is not None:
        val = val + (U * gU).sum()
    if gV is not None:
        val = val + (V * gV).sum()
    return val


def gradient(A: np.ndarray, k: int, l: int, i: int, G: np.ndarray, center: bool = False,
             gS=None, gU=None, gV=None) -> np.ndarray:
    """dL/dA (m x n float64) for L = <gS, S> + <gU, U> + <gV, V> with G fixed."""
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Gt = torch.tensor(np.asarray(G, dtype=np.float64))
    t = lambda x: None if x is None else torch.tensor(np.asarray(x, dtype=np.float64))
    U, S, V = forward(At, k, l, i, Gt, center)
    loss_value(U, S, V, t(gS), t(gU), t(gV)).backward()
    return At.grad.numpy()


def loss(A: np.ndarray, k: int, l: int, i: int, G: np.ndarray, center: bool = False,
         gS=None, gU=None, gV=None) -> float:
    """The scalar loss itself (for finite differences)."""
    with torch.no_grad():
        At = torch.tensor(np.asarray(A, dtype=np.float64))
        Gt = torch.tensor(np.asarray(G, dtype=np.float64))
        t = lambda x: None if x is None else torch.tensor(np.asarray(x, dtype=np.float64))
        U, S, V = forward(At, k, l, i, Gt, center)
        return float(loss_value(U, S, V, t(gS), t(gU), t(gV)))
