"""Low-precision storage of A (bfloat16, FP8 e4m3 with column scales, bfloat16 hi + lo).

The stored matrix is the matrix: the oracle factors the float64 values that
the reference definitions in oracle/quantize_ref.py give for the same float32
input, with the same G, and the GPU path must agree with it.  Its products
carry the float32 operand as a bfloat16 hi + lo pair (relative representation
error <= 2^-17) and accumulate in float32, so the bar is the float32 one:
singular values within 1e-5 relative, leading vectors within 1e-4.  The error
of each format against the factorisation of the float32 matrix itself is a
property of the format, printed, and checked against Weyl's bound
|sigma_j(A_q) - sigma_j(A)| <= ||A - A_q||_2.
"""
import ctypes
import os

import numpy as np
import pytest

from synth import fixtures as F
from oracle import rpca_oracle as O
from oracle import quantize_ref as Qr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIBDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_5510_amd")
STORAGES = ["bf16", "fp8_e4m3", "bf16_hilo"]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(os.path.join(LIBDIR, "librpca.so")):
        pytest.fail("librpca.so is not built (the GPU path has no fallback)")


def _np_bits(t):
    return t.cpu().numpy().view(np.uint16) if t.dtype == torch.int16 else t.cpu().numpy()


def _quantize_gpu(A, storage, shift=None, ld=None):
    from paper_1007_5510_amd import rpca
    Ad = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    sh = shift
    if isinstance(shift, np.ndarray):
        sh = torch.from_numpy(shift.astype(np.float32)).cuda()
    st = rpca.quantize(Ad, storage, shift=sh, ld=ld)
    torch.cuda.synchronize()
    return st


def _dequant_ref(A, storage, shift=None):
    data, scale = Qr.quantize(storage, A, shift)
    return Qr.dequantize(storage, data, scale)


def _run(stored, k, l, i, G, center=False, flags=0):
    from paper_1007_5510_amd import rpca, _lib
    p = rpca.Plan(stored.m, stored.n, k, l, i, storage=stored.storage, center=center,
                  flags=flags | _lib.FLAG_KEEP_STATE | _lib.FLAG_PROFILE)
    Gd = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda()
    U, S, V = p.factor(stored, G=Gd)
    torch.cuda.synchronize()
    return U.cpu().double().numpy(), S.cpu().double().numpy(), V.cpu().double().numpy(), p


def _compare(g, orc, k, s_tol=1e-5, v_tol=1e-4, n_vec=None):
    U, S, V, _ = g
    rel = np.abs(S - orc.S) / orc.S
    print(f"  sigma rel err vs oracle on stored values: {rel.max():.3e}")
    assert rel.max() <= s_tol
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-5
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-5
    nv = n_vec or k
    du = np.linalg.norm(U[:, :nv] - orc.U[:, :nv], axis=0).max()
    dv = np.linalg.norm(V[:, :nv] - orc.V[:, :nv], axis=0).max()
    print(f"  vector err U {du:.3e} V {dv:.3e}")
    assert du <= v_tol and dv <= v_tol


# ---------------------------------------------------------------- quantiser, bit for bit
def _quant_input(seed, m, n):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) * rng.uniform(0.01, 30.0, n)[None, :]).astype(np.float32)
    A[:, 3] = 0.0                                           # zero column: scale 1
    A[:, 5] = (rng.standard_normal(m) * 1e-4).astype(np.float32)
    A[7, 5] = 10.0                                          # mostly FP8 subnormal codes in column 5
    A[:, 6] += np.float32(0.5)                              # a large column mean
    A[11, :] = np.float32(1.0 + 2.0 ** -8)                  # bf16 ties
    return A


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("mode", ["none", "given", "mean"])
def test_quantize_bit_exact(storage, mode):
    _need_gpu()
    m, n = 301, 70
    A = _quant_input(5, m, n)
    shift = None
    if mode == "given":
        shift = np.linspace(-1.0, 1.0, n).astype(np.float32)
    st = _quantize_gpu(A, storage, shift=(shift if mode == "given" else ("mean" if mode == "mean" else None)))
    if mode == "mean":
        got_shift = st.shift.cpu().numpy()
        mu32 = A.astype(np.float64).mean(axis=0).astype(np.float32)
        # float64 sums in another order: equal after rounding to float32 but for a
        # rounding boundary (checked to one float32 ulp)
        assert np.all(np.abs(got_shift - mu32) <= np.spacing(np.abs(mu32)))
        shift = got_shift
    data, scale = Qr.quantize(storage, A, shift)
    ld = st.ld
    if storage == "bf16_hilo":
        got = _np_bits(st.data)
        assert np.array_equal(got[0, :, :n], data[0]) and np.array_equal(got[1, :, :n], data[1])
        assert not got[:, :, n:].any()
    else:
        got = _np_bits(st.data)
        assert np.array_equal(got[:, :n], data)
        assert not got[:, n:].any()
    if storage == "fp8_e4m3":
        assert np.array_equal(st.col_scale.cpu().numpy(), scale)
        assert not np.any(got == 0x7F) and not np.any(got == 0xFF)
    assert ld % 16 == 0


# ---------------------------------------------------------------- factorisation parity
@pytest.mark.parametrize("storage", STORAGES)
def test_lowp_plain_small(storage):
    """2000 x 1000, sigma_j = 0.9^(j-1), k=10, l=12, i=1 on each stored format: parity with the
    oracle on the stored values, and the format's error against the oracle on the float32 data."""
    _need_gpu()
    p = F.plain_small()
    A32 = p["A"].astype(np.float32)
    Aq = _dequant_ref(A32, storage)
    orc = O.rpca(Aq, p["k"], p["l"], p["i"], p["G"])
    st = _quantize_gpu(A32, storage)
    g = _run(st, p["k"], p["l"], p["i"], p["G"])
    _compare(g, orc, p["k"])
    # the format's own error against the float32 matrix (reported; Weyl envelope)
    orc32 = O.rpca(A32.astype(np.float64), p["k"], p["l"], p["i"], p["G"])
    dnorm = np.linalg.norm(Aq - A32.astype(np.float64), 2)
    sq = np.linalg.svd(Aq, compute_uv=False)
    s32 = np.linalg.svd(A32.astype(np.float64), compute_uv=False)
    assert np.abs(sq - s32).max() <= dnorm * (1 + 1e-9)
    # against the float64 oracle on the float32 data: each singular value moves by at most
    # ||A - A_q||_2 (Weyl, for the same subspace) plus the float32 arithmetic of the products
    # (1e-5 relative, twice for the two runs), and the residual meets the gate
    dS = np.abs(g[1] - orc32.S)
    rel32 = dS / orc32.S
    res = O.residual_exact(A32.astype(np.float64), g[0], g[1], g[2])
    print(f"  {storage}: sigma rel err vs float32 data {rel32.max():.3e}, max |dS| {dS.max():.3e}, "
          f"||A-A_q||_2 {dnorm:.3e}, residual/sigma_11 {res / 0.9 ** 10:.5f}")
    assert np.all(dS <= dnorm + 2e-5 * orc32.S[0])
    assert res / 0.9 ** 10 <= 1.1
    stats = g[3].stats()
    assert stats["passes"] == p["i"] + 2


@pytest.mark.parametrize("storage", STORAGES)
def test_lowp_ragged_centered(storage):
    """Ragged m, n (n not a multiple of 16 or 64), several Z tiles, centring of a shifted copy."""
    _need_gpu()
    m, n, k, l, i = 3001, 517, 6, 40, 2
    rng = np.random.default_rng(11)
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    prob = F.svd_problem(3001, m, n, sigma)
    A32 = (prob["A"] + rng.uniform(0, 1, n)[None, :]).astype(np.float32)  # column means ~U(0,1)
    G = F.gaussian_G(3001, n, l)
    st = _quantize_gpu(A32, storage, shift="mean")
    shift = st.shift.cpu().numpy()
    Aq = _dequant_ref(A32, storage, shift)
    orc = O.rpca(Aq, k, l, i, G, center=True)
    g = _run(st, k, l, i, G, center=True)
    _compare(g, orc, k, n_vec=4)
    # the column sums come from pass 0's adjoint (an implicit ones column: float32 chains per row
    # split, float64 across splits), the accumulation of the float32-storage path, same bound
    mu = g[3].state("MU").cpu().numpy()
    assert np.abs(mu - Aq.mean(axis=0)).max() <= 1e-9 * np.abs(Aq).max()


@pytest.mark.parametrize("storage", STORAGES)
def test_lowp_padding_ignored(storage):
    """Entries between n and lda are not data: NaN bit patterns there change nothing."""
    _need_gpu()
    m, n, k, l, i = 1203, 301, 5, 9, 1
    sigma = 0.85 ** np.arange(n, dtype=np.float64)
    prob = F.svd_problem(77, m, n, sigma)
    A32 = prob["A"].astype(np.float32)
    G = F.gaussian_G(77, n, l)
    st = _quantize_gpu(A32, storage, ld=336)
    nan = 0x7F if storage == "fp8_e4m3" else 0x7FC0
    st.data[..., n:] = nan
    Aq = _dequant_ref(A32, storage)
    orc = O.rpca(Aq, k, l, i, G)
    g = _run(st, k, l, i, G)
    _compare(g, orc, k)


def test_lowp_intermediates_bf16():
    """H blocks of the bfloat16 path against the oracle's on the stored values."""
    _need_gpu()
    p = F.plain_small(seed=77, m=1500, n=700)
    k, l, i = 8, 10, 2
    G = F.gaussian_G(77, 700, l)
    A32 = p["A"].astype(np.float32)
    Aq = _dequant_ref(A32, "bf16")
    orc = O.rpca(Aq, k, l, i, G)
    g = _run(_quantize_gpu(A32, "bf16"), k, l, i, G)
    plan = g[3]
    H = plan.state("H").cpu().double().numpy()
    scale = np.cumprod(plan.state("HSCALE").cpu().numpy())
    for j in range(i + 1):
        Hj = H[:, j * l:(j + 1) * l] / scale[j]
        ref = orc.H_blocks[j]
        err = np.linalg.norm(Hj - ref) / np.linalg.norm(ref)
        print(f"  H^({j}) rel err {err:.3e}")
        assert err < 2e-5
    sig = plan.state("SIGMA").cpu().numpy()
    assert (np.abs(sig[:k] - orc.Stilde[:k]) / orc.Stilde[:k]).max() < 1e-5


def test_lowp_invalid_arguments():
    _need_gpu()
    from paper_1007_5510_amd import rpca, _lib
    lib = _lib.load()
    m, n = 256, 64
    A = torch.randn(m, n, device="cuda")
    out = torch.zeros(m, 72, dtype=torch.int16, device="cuda")
    P = _lib.PANEL_CB()
    # ldo not a multiple of 16
    rc = lib.rpca_quantize(1, m, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), 72,
                           None, None, 0, None)
    assert rc == 1
    # F32 is not a quantised format; FP8 needs col_scale; bad shift mode
    rc = lib.rpca_quantize(0, m, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), 64,
                           None, None, 0, None)
    assert rc == 1
    rc = lib.rpca_quantize(2, m, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), 64,
                           None, None, 0, None)
    assert rc == 1
    rc = lib.rpca_quantize(1, m, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), 64,
                           None, None, 1, None)
    assert rc == 1
    # factor: lda % 16 != 0, and FP8 without scales
    p = rpca.Plan(m, n, 4, 6, 1, storage="bf16")
    U = torch.empty(m, 4, device="cuda")
    S = torch.empty(4, device="cuda")
    V = torch.empty(n, 4, device="cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = lib.rpca_factor(p.handle, ptr(out), 72, None, P, None, None, ptr(U), 4, ptr(S), ptr(V), 4)
    assert rc == 1
    p8 = rpca.Plan(m, n, 4, 6, 1, storage="fp8_e4m3")
    q8 = torch.zeros(m, 64, dtype=torch.uint8, device="cuda")
    rc = lib.rpca_factor(p8.handle, ptr(q8), 64, None, P, None, None, ptr(U), 4, ptr(S), ptr(V), 4)
    assert rc == 1
