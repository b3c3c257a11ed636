"""GPU path vs the float64 oracle on the same seeded inputs (through the C ABI).

Tolerances follow from float32 storage and float32 matrix-core products with
float64 QR and small eigensolver: singular values within 1e-5 relative (the
float32 target), singular vectors (clear gaps only) within 1e-4 in 2-norm,
outputs orthonormal to 1e-5, and the residual gate ||A~ - U S V^T|| / sigma_{k+1}
<= 1.1.
"""
import math
import os

import numpy as np
import pytest

from synth import fixtures as F
from oracle import rpca_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIBDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_5510_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(os.path.join(LIBDIR, "librpca.so")):
        pytest.fail("librpca.so is not built (the GPU path has no fallback)")


def run_gpu(A, k, l, i, G=None, center=False, flags=0, lda=None, seed=0):
    """Upload A (float32, host) with leading dimension lda and factor it on cuda:0."""
    _need_gpu()
    from paper_1007_5510_amd import rpca
    from paper_1007_5510_amd import _lib
    m, n = A.shape
    lda = lda or n
    buf = torch.zeros((m, lda), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    Ad = buf[:, :n]
    Gd = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda() if G is not None else None
    p = rpca.Plan(m, n, k, l, i, center=center, seed=seed,
                  flags=flags | _lib.FLAG_KEEP_STATE | _lib.FLAG_PROFILE)
    U, S, V = p.factor(Ad, G=Gd)
    torch.cuda.synchronize()
    return (U.cpu().double().numpy(), S.cpu().double().numpy(), V.cpu().double().numpy(), p)


def compare(gpu, orc, k, gap_vectors=True, s_tol=1e-5, v_tol=1e-4, n_vec=None):
    """n_vec: compare only the leading n_vec singular vectors (those with clear gaps)."""
    U, S, V, _ = gpu
    rel = np.abs(S - orc.S) / orc.S
    print(f"  sigma rel err max {rel.max():.3e}")
    assert rel.max() <= s_tol
    assert np.all(np.diff(S) <= 1e-6 * S[0])
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-5
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-5
    if gap_vectors:
        nv = n_vec or k
        du = np.linalg.norm(U[:, :nv] - orc.U[:, :nv], axis=0).max()
        dv = np.linalg.norm(V[:, :nv] - orc.V[:, :nv], axis=0).max()
        print(f"  vector err max U {du:.3e} V {dv:.3e}")
        assert du <= v_tol and dv <= v_tol


def test_plain_small_parity():
    """2000 x 1000, sigma_j = 0.9^(j-1), k=10, l=12, i=1, no centring."""
    p = F.plain_small()
    orc = O.rpca(p["A"], p["k"], p["l"], p["i"], p["G"])
    g = run_gpu(p["A"], p["k"], p["l"], p["i"], G=p["G"])
    compare(g, orc, p["k"])
    U, S, V, plan = g
    res = O.residual_exact(p["A"], U, S, V)
    assert res / 0.9 ** 10 <= 1.1
    st = plan.stats()
    assert st["passes"] == p["i"] + 2
    assert st["qr_fallback"] == 0


def test_intermediates_match_oracle():
    """H blocks (up to the positive block scales), span(Q), and the Ritz values S~ of Step 4."""
    p = F.plain_small(seed=77, m=1500, n=700)
    k, l, i = 8, 10, 2
    G = F.gaussian_G(77, 700, l)
    orc = O.rpca(p["A"], k, l, i, G)
    U, S, V, plan = run_gpu(p["A"], k, l, i, G=G)
    H = plan.state("H").cpu().double().numpy()
    scale = np.cumprod(plan.state("HSCALE").cpu().numpy())
    for j in range(i + 1):
        Hj = H[:, j * l:(j + 1) * l] / scale[j]
        ref = orc.H_blocks[j]
        err = np.linalg.norm(Hj - ref) / np.linalg.norm(ref)
        print(f"  H^({j}) rel err {err:.3e}")
        assert err < 2e-6
    Q = plan.state("Q").cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye((i + 1) * l)).max() < 1e-12
    Pg = Q @ (Q.T @ orc.Q[:, :k])  # projection of the oracle's leading basis onto span(Q_gpu)
    assert np.linalg.norm(Pg - orc.Q[:, :k]) < 1e-4
    sig = plan.state("SIGMA").cpu().numpy()
    rel = np.abs(sig[:k] - orc.Stilde[:k]) / orc.Stilde[:k]
    assert rel.max() < 1e-5
    T = plan.state("T").cpu().numpy()
    st = np.linalg.svd(T, compute_uv=False)
    assert np.abs(st[:k] - orc.Stilde[:k]).max() / orc.Stilde[0] < 1e-5
    # Step 4 on the device's own T: every eigenpair of T^T T (state keeps all L)
    L = (i + 1) * l
    Mg = T.T @ T
    ev = np.sort(np.linalg.eigvalsh(Mg))[::-1]
    sig_all = plan.state("SIGMA").cpu().numpy()
    assert np.abs(sig_all ** 2 - ev).max() < 1e-12 * ev[0]
    Wg = plan.state("W").cpu().numpy()
    assert np.abs(Wg.T @ Wg - np.eye(L)).max() < 1e-10
    assert np.linalg.norm(Mg @ Wg - Wg * ev) < 1e-11 * ev[0]


@pytest.mark.parametrize("m,n,k,l,i,lda,v_tol", [
    (1037, 333, 5, 7, 2, None, 1e-4),     # ragged everything, lda % 4 != 0 (scalar loads)
    (1037, 333, 5, 7, 2, 336, 1e-4),      # same data, padded lda (vector loads)
    (777, 200, 1, 1, 3, None, 1e-4),      # l = 1
    (900, 300, 6, 8, 0, None, 1e-4),      # i = 0: the basic randomized SVD
    # L = 120 and L = 210 with sigma_j = 0.93^(j-1): the last power block has
    # condition ~ (sigma_1/sigma_L)^5 > 1/u, so the trailing directions of span(Q)
    # are fixed by rounding on both sides; the leading vectors inherit ~1e-3
    # while the singular values stay at ~1e-7 (second order).
    (4000, 1500, 30, 40, 2, None, 2e-3),  # several Z tiles, 2 Gram tiles, block Jacobi
    (5000, 1200, 40, 70, 2, None, 2e-3),  # Cholesky / inverse in global memory
])
def test_shapes_and_edges(m, n, k, l, i, lda, v_tol):
    sigma = 0.93 ** np.arange(n, dtype=np.float64)
    p = F.svd_problem(1000 + m, m, n, sigma)
    G = F.gaussian_G(1000 + m, n, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G, lda=lda)
    compare(g, orc, k, v_tol=v_tol)
    # the approximation is as good as the oracle's: same spectral residual to 1e-5
    r_g = O.residual_exact(p["A"], g[0], g[1], g[2])
    r_o = O.residual_exact(p["A"], orc.U, orc.S, orc.V)
    print(f"  residual gpu {r_g:.6e} oracle {r_o:.6e}  fallback {g[3].stats()['qr_fallback']}")
    assert abs(r_g - r_o) / r_o < 1e-5


def test_centered_parity():
    """Low-rank + noise + U(0,1) column offsets, centred (the in-core structure at small size)."""
    m, n, r = 6000, 800, 12
    sig = 1.0 / np.arange(1, r + 1)
    p = F.lowrank_noise(31, m, n, r, sig, 1e-3, True)
    k, l, i = 10, 14, 2
    G = F.gaussian_G(31, n, l)
    orc = O.rpca(p["A"], k, l, i, G, center=True)
    g = run_gpu(p["A"], k, l, i, G=G, center=True)
    # Ritz values 5..10 sit in the noise bulk (noise norm ~0.1): their vectors have no
    # clear gap, so vectors are compared for the 4 signal directions only.
    compare(g, orc, k, n_vec=4)
    U, S, V, plan = g
    # the column means are folded into pass 0: mu = s0 + colsum(A - 1 s0^T) / m, the deviation sums
    # accumulated on float32 matrix cores (one float32 chain per row split) and in float64 across splits
    mu = plan.state("MU").cpu().numpy()
    assert np.abs(mu - orc.mu).max() < 1e-9 * np.abs(p["A"]).max()
    assert np.abs(np.ones(m) @ U).max() < 1e-4


def test_generated_G_matches_generator():
    """G drawn inside the library from the seed equals the seeded generator's G (to rounding)."""
    p = F.plain_small(seed=5, m=1200, n=500)
    k, l, i, seed = 6, 8, 1, 424242
    G = F.gaussian_G(seed, 500, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=None, seed=seed)
    compare(g, orc, k)


def test_forced_fallback_agrees():
    from paper_1007_5510_amd import _lib
    p = F.plain_small(seed=6, m=1500, n=600)
    k, l, i = 8, 10, 1
    G = F.gaussian_G(6, 600, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G, flags=_lib.FLAG_FORCE_FALLBACK)
    compare(g, orc, k)
    assert g[3].stats()["qr_fallback"] == 1


def test_rank_deficient_takes_fallback():
    """rank(A) = 5 < (i+1) l: H is numerically rank deficient; the exact SVD comes back."""
    m, n = 800, 300
    sigma = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    U0 = F.haar(9, F.STREAM_U, m, 5)
    V0 = F.haar(9, F.STREAM_V, n, 5)
    A = F.to_f32((U0 * sigma) @ V0.T)
    G = F.gaussian_G(9, n, 6)
    U, S, V, plan = run_gpu(A, 4, 6, 1, G=G)
    print(f"  fallback taken: {plan.stats()['qr_fallback']}")
    assert np.abs(S - sigma[:4]).max() / 5.0 < 1e-5
    res = O.residual_exact(A, U, S, V)
    assert abs(res - 0.5) < 1e-5


def test_deterministic_repeat():
    p = F.plain_small(seed=12, m=3000, n=900)
    G = F.gaussian_G(12, 900, 12)
    a = run_gpu(p["A"], 10, 12, 2, G=G)
    b = run_gpu(p["A"], 10, 12, 2, G=G)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_nonfinite_is_reported():
    from paper_1007_5510_amd import rpca, _lib
    _need_gpu()
    A = F.plain_small(seed=3, m=500, n=200)["A"].copy()
    A[17, 33] = np.nan
    Ad = torch.from_numpy(A).cuda()
    with rpca.Plan(500, 200, 5, 6, 1) as p:
        with pytest.raises(_lib.RPCAError) as e:
            p.factor(Ad)
        assert e.value.code == 6


def test_invalid_arguments_on_device():
    from paper_1007_5510_amd import rpca, _lib
    _need_gpu()
    with pytest.raises(_lib.RPCAError) as e:
        rpca.Plan(500, 200, 10, 8, 1)
    assert e.value.code == 1
    with rpca.Plan(500, 200, 5, 6, 1) as p:
        with pytest.raises(_lib.RPCAError):
            p.state("H")  # nothing kept yet


def test_householder_step2_parity():
    """Step 2 by the Householder TSQR (forced): the same factorisation as the oracle, Q orthonormal to
    float64 rounding, Q R = H with the returned triangle (through the reverse sweep's use of R below)."""
    from paper_1007_5510_amd import _lib
    p = F.plain_small(seed=8, m=3000, n=900)
    k, l, i = 10, 14, 2
    G = F.gaussian_G(8, 900, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G, flags=_lib.FLAG_FORCE_HOUSEHOLDER)
    compare(g, orc, k)
    plan = g[3]
    assert plan.stats()["qr_fallback"] == 3
    Q = plan.state("Q").cpu().numpy()
    L = (i + 1) * l
    assert np.abs(Q.T @ Q - np.eye(L)).max() < 1e-13
    H = plan.state("H").cpu().double().numpy()
    Pq = Q @ (Q.T @ H)  # span(Q) = span(H)
    assert np.linalg.norm(Pq - H) < 1e-12 * np.linalg.norm(H)


def test_householder_step2_centered_and_rank_deficient():
    from paper_1007_5510_amd import _lib
    m, n, r = 6000, 800, 12
    sig = 1.0 / np.arange(1, r + 1)
    p = F.lowrank_noise(31, m, n, r, sig, 1e-3, True)
    k, l, i = 10, 14, 2
    G = F.gaussian_G(31, n, l)
    orc = O.rpca(p["A"], k, l, i, G, center=True)
    g = run_gpu(p["A"], k, l, i, G=G, center=True, flags=_lib.FLAG_FORCE_HOUSEHOLDER)
    compare(g, orc, k, n_vec=4)
    assert g[3].stats()["qr_fallback"] == 3
    # rank(A) = 5 < L = 12: H numerically rank deficient, Householder completes Q
    m, n = 800, 300
    sigma = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    U0 = F.haar(9, F.STREAM_U, m, 5)
    V0 = F.haar(9, F.STREAM_V, n, 5)
    A = F.to_f32((U0 * sigma) @ V0.T)
    U, S, V, plan = run_gpu(A, 4, 6, 1, G=F.gaussian_G(9, n, 6), flags=_lib.FLAG_FORCE_HOUSEHOLDER)
    assert plan.stats()["qr_fallback"] == 3
    assert np.abs(S - sigma[:4]).max() / 5.0 < 1e-5
    assert abs(O.residual_exact(A, U, S, V) - 0.5) < 1e-5


def test_block_rescale_keeps_large_matrices_finite():
    """Section 3's overflow remark: with ||A|| = 1e10 and i = 3 the unscaled powers reach ~1e70,
    far past float32; the positive block rescale keeps every iterate finite and the factorisation
    scales exactly, while RPCA_FLAG_NO_RESCALE reports the overflow.  (A block X_j enters its
    forward product before its scale, so the float32 path needs ||A||^3 well inside float32.)"""
    from paper_1007_5510_amd import _lib
    p = F.plain_small(seed=21, m=2000, n=1000)
    A = F.to_f32(p["A"].astype(np.float64) * 1e10)
    k, l, i = 8, 10, 3
    G = F.gaussian_G(21, 1000, l)
    orc = O.rpca(A, k, l, i, G)
    g = run_gpu(A, k, l, i, G=G)
    compare(g, orc, k)
    assert np.all(np.isfinite(g[0])) and np.all(np.isfinite(g[2]))
    with pytest.raises(_lib.RPCAError) as e:
        run_gpu(A, k, l, i, G=G, flags=_lib.FLAG_NO_RESCALE)
    assert e.value.code == 6  # RPCA_ERR_NONFINITE


@pytest.mark.parametrize("m,n,k,l,i", [
    (12000, 1500, 40, 64, 3),   # L = 256
    (6000, 1200, 100, 120, 2),  # L = 360, the width of the streamed workload (k = 100, l = 120, i = 2)
])
def test_householder_step2_wide(m, n, k, l, i):
    """Householder Step 2 forced at L = 256 and L = 360 (one workgroup per row block holds the
    block's reflector and partial sums in LDS: up to L = 1024 on gfx950): parity with the oracle's
    pivoted QR route and an orthonormal Q."""
    from paper_1007_5510_amd import _lib
    sigma = 0.97 ** np.arange(n, dtype=np.float64)
    p = F.svd_problem(7070 + l, m, n, sigma)
    G = F.gaussian_G(7070 + l, n, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G, flags=_lib.FLAG_FORCE_HOUSEHOLDER)
    assert g[3].stats()["qr_fallback"] == 3
    compare(g, orc, k, v_tol=2e-3)
    Q = g[3].state("Q").cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye((i + 1) * l)).max() < 1e-13


@pytest.mark.parametrize("m,n,k,l,i,decay,levels", [
    (12000, 1500, 40, 64, 1, 0.998, (0,)),     # L = 128: Cholesky QR twice, LDS-resident factor
    (12000, 1500, 40, 128, 1, 0.998, (0,)),    # L = 256: Cholesky QR twice, factor in global memory
    (6000, 1200, 100, 120, 2, 0.995, (0,)),    # L = 360, the width of the streamed workload
    (6000, 1200, 100, 120, 2, 0.97, (1, 2)),   # L = 360, ill-conditioned H: shifted rounds
    (8000, 2000, 100, 200, 2, 0.999, (0,)),    # L = 600: four block rows per wave in the inverse
])
def test_cholesky_qr_wide(m, n, k, l, i, decay, levels):
    """Cholesky QR (Step 2, Section 3) up to L = 600, where the Gram factor and its inverse run
    blocked in global memory (the packed triangle no longer fits in LDS): the plain rounds for a
    well-conditioned H, the shifted rounds for an ill-conditioned one; parity with the oracle's
    pivoted QR route and an orthonormal Q."""
    sigma = decay ** np.arange(n, dtype=np.float64)
    p = F.svd_problem(7170 + l, m, n, sigma)
    G = F.gaussian_G(7170 + l, n, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G)
    level = g[3].stats()["qr_fallback"]
    print(f"  L = {(i + 1) * l}: Step 2 level {level}")
    assert level in levels
    compare(g, orc, k, v_tol=2e-3)
    Q = g[3].state("Q").cpu().numpy()
    L = (i + 1) * l
    assert np.abs(Q.T @ Q - np.eye(L)).max() < 1e-13


@pytest.mark.parametrize("k,l,i", [(20, 40, 2), (16, 24, 2), (20, 44, 1), (50, 60, 2)])
def test_wide_t_pass_matches_fallback_bitwise(k, l, i):
    """The T pass with L = 120 (8 tiles of 16 columns), 180 (12 tiles), 72 or 88 (6 tiles, 8-byte Z
    pieces) runs on the wide-Z adjoint when A's rows allow vector loads and on the 64-column adjoint
    otherwise; both sum every output over the same rows in the same order, so the same matrix with an
    aligned and with an odd leading dimension factors to identical bits."""
    m, n = 6000, 1000
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    p = F.svd_problem(6100, m, n, sigma)
    G = F.gaussian_G(6100, n, l)
    a = run_gpu(p["A"], k, l, i, G=G, lda=1004)  # 16-byte rows: vector loads, wide T pass
    b = run_gpu(p["A"], k, l, i, G=G, lda=1001)  # odd stride: scalar loads, 64-column T pass
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[3].state("T").cpu().numpy(), b[3].state("T").cpu().numpy())
