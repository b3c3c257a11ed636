"""Python surface of the library: the C-ABI calls with torch tensors for device memory.

Every step of the method runs inside librpca.so; this module only checks
tensor properties, allocates outputs with torch and passes raw pointers and
the current HIP stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, load, Desc, Stats, STORAGE, SOURCE, STATE, PANEL_CB, DEVICE_PANEL_CB

_STATE_DTYPE = {"H": torch.float32}
_STORED_DTYPE = {"bf16": torch.int16, "bf16_hilo": torch.int16, "fp8_e4m3": torch.uint8}


class Stored:
    """A matrix in one of the library's stored formats (output of :func:`quantize`).

    data: bf16 -> int16 (m, ld) bit patterns; bf16_hilo -> int16 (2, m, ld) (hi plane, lo plane);
    fp8_e4m3 -> uint8 (m, ld) codes with col_scale (n,) float32.  shift (n,) float32 or None is
    the per-column value subtracted before conversion.
    """

    def __init__(self, storage, data, m, n, col_scale=None, shift=None):
        self.storage, self.data, self.m, self.n = storage, data, int(m), int(n)
        self.col_scale, self.shift = col_scale, shift
        self.ld = data.stride(-2)


def quantize(A, storage, shift=None, ld=None):
    """Convert a float32 device matrix with rpca_quantize.

    shift: None (no shift), "mean" (column means computed by the library), or an (n,) float32 tensor.
    """
    lib = load()
    if A.dtype != torch.float32 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a row-major 2-D float32 tensor")
    m, n = A.shape
    ld = int(ld) if ld is not None else (n + 15) // 16 * 16
    dt = _STORED_DTYPE[storage]
    shape = (2, m, ld) if storage == "bf16_hilo" else (m, ld)
    data = torch.empty(shape, dtype=dt, device=A.device)
    col_scale = torch.empty((n,), dtype=torch.float32, device=A.device) if storage == "fp8_e4m3" else None
    if shift is None:
        mode, sh = 0, None
    elif isinstance(shift, str):
        if shift != "mean":
            raise ValueError("shift must be None, 'mean' or a tensor")
        mode, sh = 2, torch.empty((n,), dtype=torch.float32, device=A.device)
    else:
        if shift.dtype != torch.float32 or tuple(shift.shape) != (n,) or not shift.is_contiguous():
            raise ValueError(f"shift must be a contiguous float32 ({n},) tensor")
        mode, sh = 1, shift
    check(lib.rpca_quantize(STORAGE[storage], m, n, _ptr(A), A.stride(0), _ptr(data), ld, _ptr(col_scale),
                            _ptr(sh), mode, _stream(A.device)), "rpca_quantize")
    return Stored(storage, data, m, n, col_scale=col_scale, shift=sh)


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
        self.source = source
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

    def factor(self, A=None, G=None, col_scale=None, out=None, panel_fn=None):
        """A: a float32 row-major tensor (f32 plans) or a :class:`Stored` from :func:`quantize`.

        source "host_pinned": A is a pinned CPU float32 tensor.  source "callback": A is None and
        panel_fn(row0, nrows, buf) fills buf[:, :n] (a float32 NumPy view of nrows x ld, pinned host
        memory) with rows row0 .. row0 + nrows - 1 and returns nothing (an exception is reported as
        RPCA_ERR_CALLBACK).  source "device_callback": A is None and panel_fn(row0, nrows, dst, ld,
        stream) enqueues on the HIP stream `stream` (an integer handle) device work writing those rows
        as float32 to the device address `dst` (leading dimension ld) and returns nothing.
        """
        m, n, k = self.m, self.n, self.k
        cb = PANEL_CB()
        data, lda = None, 0
        if self.source == "device_callback":
            if panel_fn is None:
                raise ValueError("a device_callback plan needs panel_fn")

            def _dcb(user, row0, nrows, dst, ld, stream):
                try:
                    panel_fn(int(row0), int(nrows), int(dst), int(ld), int(stream or 0))
                    return 0
                except Exception:
                    return 1
            self._dcb = DEVICE_PANEL_CB(_dcb)  # kept alive with the plan
            check(self.lib.rpca_set_device_panel_cb(self.handle, self._dcb, None), "rpca_set_device_panel_cb")
        elif self.source == "callback":
            if panel_fn is None:
                raise ValueError("a callback plan needs panel_fn")
            import numpy as np

            def _cb(user, row0, nrows, dst, ld, cs):
                try:
                    buf = np.ctypeslib.as_array(ctypes.cast(dst, ctypes.POINTER(ctypes.c_float)),
                                                shape=(int(nrows), int(ld)))
                    panel_fn(int(row0), int(nrows), buf)
                    return 0
                except Exception:
                    return 1
            cb = PANEL_CB(_cb)
        elif self.source == "host_pinned":
            if A.device.type != "cpu" or not A.is_pinned() or A.dtype != torch.float32 or A.stride(1) != 1:
                raise ValueError("a host_pinned plan takes a pinned CPU float32 row-major tensor")
            data, lda = A, A.stride(0)
        elif isinstance(A, Stored):
            if A.storage != self.storage or A.m != m or A.n != n:
                raise ValueError(f"stored matrix is {A.storage} {A.m} x {A.n}; plan is {self.storage} {m} x {n}")
            data, lda, col_scale = A.data, A.ld, A.col_scale
        else:
            if self.storage != "f32":
                raise ValueError("a low-precision plan takes the Stored result of quantize()")
            if A.dim() != 2 or A.shape[0] < m or A.stride(1) != 1 or A.dtype != torch.float32:
                raise ValueError("A must be a row-major 2-D float32 tensor")
            data, lda = A, A.stride(0)
        if self.source == "device" and data.device != self.device:
            raise ValueError("A must live on the plan's device")
        if G is not None:
            gn = min(m, n)  # m < n: the test matrix of A^T's problem
            if G.dtype != torch.float32 or tuple(G.shape) != (gn, self.l) or not G.is_contiguous():
                raise ValueError(f"G must be a contiguous float32 {gn} x {self.l} tensor")
        if out is None:
            U = torch.empty((m, k), dtype=torch.float32, device=self.device)
            S = torch.empty((k,), dtype=torch.float32, device=self.device)
            V = torch.empty((n, k), dtype=torch.float32, device=self.device)
        else:
            U, S, V = out
        rc = self.lib.rpca_factor(self.handle, _ptr(data), lda, _ptr(col_scale), cb, None, _ptr(G),
                                  _ptr(U), U.stride(0), _ptr(S), _ptr(V), V.stride(0))
        check(rc, "rpca_factor")
        return U, S, V

    def backward(self, gS=None, gU=None, gV=None, out=None):
        """dL/dA for L = <gS, S> + <gU, U> + <gV, V> after a factor() with FLAG_KEEP_STATE (G held fixed)."""
        m, n, k = self.m, self.n, self.k
        for name, t, shape in (("gS", gS, (k,)), ("gU", gU, (m, k)), ("gV", gV, (n, k))):
            if t is not None and (t.dtype != torch.float32 or tuple(t.shape) != shape or t.stride(-1) != 1
                                  or t.device != self.device):
                raise ValueError(f"{name} must be a float32 {shape} tensor on the plan's device")
        dA = out if out is not None else torch.empty((m, n), dtype=torch.float32, device=self.device)
        check(self.lib.rpca_backward(self.handle, _ptr(gS), _ptr(gU), gU.stride(0) if gU is not None else 0,
                                     _ptr(gV), gV.stride(0) if gV is not None else 0, _ptr(dA), dA.stride(0)),
              "rpca_backward")
        return dA

    def residual(self, A, U, S, V, j=6, q=None, seed=0):
        """Appendix estimate p_{j,q} of ||A~ - U S V^T||_2 (q start vectors, default k; device float32 inputs)."""
        q = self.k if q is None else int(q)
        est = ctypes.c_double(0.0)
        check(self.lib.rpca_residual(self.handle, _ptr(A), A.stride(0), None, _ptr(U), U.stride(0), _ptr(S), _ptr(V),
                                     V.stride(0), int(j), q, int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(est)),
              "rpca_residual")
        return est.value

    def state(self, which: str):
        m, n, L = self.m, self.n, self.L
        shapes = {"H": ((m, L), torch.float32), "H64": ((m, L), torch.float64), "HSCALE": ((self.i + 1,), torch.float64),
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
    """One-shot rank-k randomized PCA of the device matrix A (m x n; m < n runs on A^T)."""
    m, n = A.shape
    with Plan(m, n, k, l, i, center=center, seed=seed, flags=flags, device=A.device) as p:
        return p.factor(A, G=G)


class _RPCAFunction(torch.autograd.Function):
    """(U, S, V) = rpca(A) with the library's reverse sweep as the backward (G fixed)."""

    @staticmethod
    def forward(ctx, A, plan, G):
        U, S, V = plan.factor(A, G=G)
        ctx.plan = plan
        return U, S, V

    @staticmethod
    def backward(ctx, gU, gS, gV):
        c = lambda t: None if t is None else t.contiguous()
        dA = ctx.plan.backward(gS=c(gS), gU=c(gU), gV=c(gV))
        return dA, None, None


def rpca_autograd(A, k, l, i, *, center=False, G=None, seed=0):
    """Differentiable randomized PCA of a float32 device matrix: returns (U, S, V) with autograd support.

    The plan (holding the forward state the backward needs) lives as long as the returned tensors' graph.
    """
    m, n = A.shape
    plan = Plan(m, n, k, l, i, center=center, seed=seed, flags=_lib.FLAG_KEEP_STATE, device=A.device)
    return _RPCAFunction.apply(A, plan, G)
