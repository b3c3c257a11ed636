"""Python surface of the library: the C-ABI calls with torch tensors for device memory.

Every step of the method runs inside librpca.so; this module only checks
tensor properties, allocates outputs with torch and passes raw pointers and
the current HIP stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, load, Desc, Stats, STORAGE, SOURCE, STATE, PANEL_CB

_STATE_DTYPE = {"H": torch.float32}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A planned factorisation of an m x n matrix: rank k, block width l, i power steps.

    ``factor(A, G=None)`` returns (U, S, V) as float32 tensors on A's device.
    """

    def __init__(self, m, n, k, l, i, *, storage="f32", source="device", center=False, panel_rows=0,
                 seed=0, flags=0, device=None):
        self.lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.m, self.n, self.k, self.l, self.i = int(m), int(n), int(k), int(l), int(i)
        self.L = (self.i + 1) * self.l
        self.center = bool(center)
        self.storage = storage
        d = Desc(m=self.m, n=self.n, k=self.k, l=self.l, i=self.i, storage=STORAGE[storage],
                 source=SOURCE[source], center=1 if center else 0, panel_rows=int(panel_rows),
                 seed=int(seed) & 0xFFFFFFFFFFFFFFFF, flags=int(flags), device=self.device.index or 0)
        h = ctypes.c_void_p(0)
        check(self.lib.rpca_plan(ctypes.byref(d), _stream(self.device), ctypes.byref(h)), "rpca_plan")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.rpca_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def factor(self, A, G=None, col_scale=None, out=None):
        m, n, k = self.m, self.n, self.k
        if A.device != self.device:
            raise ValueError("A must live on the plan's device")
        if A.dim() != 2 or A.shape[0] < m or A.stride(1) != 1:
            raise ValueError("A must be a row-major 2-D tensor")
        if G is not None:
            if G.dtype != torch.float32 or tuple(G.shape) != (n, self.l) or not G.is_contiguous():
                raise ValueError(f"G must be a contiguous float32 {n} x {self.l} tensor")
        if out is None:
            U = torch.empty((m, k), dtype=torch.float32, device=self.device)
            S = torch.empty((k,), dtype=torch.float32, device=self.device)
            V = torch.empty((n, k), dtype=torch.float32, device=self.device)
        else:
            U, S, V = out
        lda = A.stride(0)
        cb = PANEL_CB()
        rc = self.lib.rpca_factor(self.handle, _ptr(A), lda, _ptr(col_scale), cb, None, _ptr(G),
                                  _ptr(U), U.stride(0), _ptr(S), _ptr(V), V.stride(0))
        check(rc, "rpca_factor")
        return U, S, V

    def state(self, which: str):
        m, n, L = self.m, self.n, self.L
        shapes = {"H": ((m, L), torch.float32), "HSCALE": ((self.i + 1,), torch.float64),
                  "Q": ((m, L), torch.float64), "T": ((n, L), torch.float64),
                  "SIGMA": ((L,), torch.float64), "W": ((L, L), torch.float64), "MU": ((n,), torch.float64)}
        shape, dt = shapes[which]
        out = torch.empty(shape, dtype=dt, device=self.device)
        ld = shape[1] if len(shape) == 2 else shape[0]
        check(self.lib.rpca_get_state(self.handle, STATE[which], _ptr(out), ld), "rpca_get_state")
        return out

    def stats(self) -> dict:
        s = Stats()
        check(self.lib.rpca_get_stats(self.handle, ctypes.byref(s)), "rpca_get_stats")
        return s.as_dict()


def factor(A, k, l, i, *, center=False, G=None, seed=0, flags=0):
    """One-shot rank-k randomized PCA of the device matrix A (m x n, m >= n)."""
    m, n = A.shape
    with Plan(m, n, k, l, i, center=center, seed=seed, flags=flags, device=A.device) as p:
        return p.factor(A, G=G)
