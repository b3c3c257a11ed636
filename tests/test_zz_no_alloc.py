"""rpca_quantize_noalloc (scratch in a fixed device array, no allocation) against rpca_quantize
(scratch allocated per call), both called through the C ABI on the same device inputs: stored
codes, column scales and computed shifts identical bit for bit, on two calls in a row with the
second one smaller (the array keeps the first call's contents)."""
import ctypes
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIBDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_5510_amd")
STORAGES = {"bf16": (1, torch.int16), "fp8_e4m3": (2, torch.uint8), "bf16_hilo": (3, torch.int16)}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(os.path.join(LIBDIR, "librpca.so")):
        pytest.fail("librpca.so is not built (the GPU path has no fallback)")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _convert(fn, storage, A, shift_mode, shift_in=None):
    code, dt = STORAGES[storage]
    m, n = A.shape
    ldo = (n + 15) // 16 * 16
    out = torch.full((2 * m if storage == "bf16_hilo" else m, ldo), 77, dtype=dt, device="cuda")
    cs = torch.full((n,), -1.0, dtype=torch.float32, device="cuda") if storage == "fp8_e4m3" else None
    if shift_mode == 2:
        sh = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    else:
        sh = shift_in
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print(f"  {fn.__name__} storage={storage} m={m} n={n} shift_mode={shift_mode}", flush=True)
    st = fn(code, m, n, _p(A), A.stride(0), _p(out), ldo, _p(cs), _p(sh), shift_mode, stream)
    torch.cuda.synchronize()
    assert st == 0, st
    return out.cpu().numpy(), (cs.cpu().numpy() if cs is not None else None), (sh.cpu().numpy() if sh is not None else None)


def _inputs(seed, m, n):
    g = torch.Generator(device="cpu").manual_seed(seed)
    A = torch.randn((m, n), generator=g, dtype=torch.float32) * 0.3 + torch.rand((n,), generator=g) * 4.0
    A[:, 3] = 0.0  # a zero column: FP8 scale 1
    A[5, :] *= 300.0  # large entries: FP8 saturation at +-448 after scaling
    return A.cuda()


@pytest.mark.parametrize("storage", ["bf16", "fp8_e4m3", "bf16_hilo"])
@pytest.mark.parametrize("shift_mode", [0, 1, 2])
def test_noalloc_matches_allocating_quantize(storage, shift_mode):
    _need_gpu()
    from paper_1007_5510_amd import _lib
    lib = _lib.load()
    # first call: 9 row splits of the column sums and maxima; second call smaller (1 split, fewer columns)
    for seed, (m, n) in ((11, (36000, 700)), (12, (3000, 300))):
        A = _inputs(seed, m, n)
        shift = (torch.rand((n,), dtype=torch.float32) * 2.0).cuda() if shift_mode == 1 else None
        ref = _convert(lib.rpca_quantize, storage, A, shift_mode, shift)
        got = _convert(lib.rpca_quantize_noalloc, storage, A, shift_mode, shift)
        for a, b in zip(ref, got):
            if a is None:
                assert b is None
            else:
                assert a.dtype == b.dtype and a.shape == b.shape
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_noalloc_scratch_limit_leaves_outputs_untouched():
    _need_gpu()
    from paper_1007_5510_amd import _lib
    lib = _lib.load()
    m, n = 1 << 20, 10896  # 256 splits: n * (12 * 256 + 8) bytes > 32 MiB
    A = torch.zeros((16, 16), dtype=torch.float32, device="cuda")  # never read: the call is refused first
    out = torch.zeros((16,), dtype=torch.int16, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.rpca_quantize_noalloc(1, m, n, _p(A), n, _p(out), n, None, None, 0, stream) == 9
