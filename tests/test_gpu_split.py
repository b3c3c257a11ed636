"""Parity of the split-operand float32 products (RPCA_FLAG_SPLIT_BF16: each float32
operand as three bfloat16 parts on the bfloat16 matrix cores) against the float64 oracle,
with the tolerances of the float32 matrix-core path."""
import numpy as np
import pytest

from oracle import rpca_oracle as O
from synth import fixtures as F
from tests.test_gpu_parity import run_gpu, compare, _need_gpu

pytestmark = pytest.mark.gpu


def _flag():
    from paper_1007_5510_amd import _lib
    return _lib.FLAG_SPLIT_BF16


def test_split_plain_small_parity():
    """2000 x 1000, sigma_j = 0.9^(j-1), k=10, l=12, i=1, no centring."""
    p = F.plain_small()
    orc = O.rpca(p["A"], p["k"], p["l"], p["i"], p["G"])
    g = run_gpu(p["A"], p["k"], p["l"], p["i"], G=p["G"], flags=_flag())
    compare(g, orc, p["k"])
    res = O.residual_exact(p["A"], g[0], g[1], g[2])
    assert res / 0.9 ** 10 <= 1.1


def test_split_intermediates_match_oracle():
    """H blocks to 2e-6 and the Ritz values of Step 4 to 1e-5, as for the float32 kernels."""
    p = F.plain_small(seed=77, m=1500, n=700)
    k, l, i = 8, 10, 2
    G = F.gaussian_G(77, 700, l)
    orc = O.rpca(p["A"], k, l, i, G)
    U, S, V, plan = run_gpu(p["A"], k, l, i, G=G, flags=_flag())
    H = plan.state("H").cpu().double().numpy()
    scale = np.cumprod(plan.state("HSCALE").cpu().numpy())
    for j in range(i + 1):
        Hj = H[:, j * l:(j + 1) * l] / scale[j]
        err = np.linalg.norm(Hj - orc.H_blocks[j]) / np.linalg.norm(orc.H_blocks[j])
        print(f"  H^({j}) rel err {err:.3e}")
        assert err < 2e-6
    sig = plan.state("SIGMA").cpu().numpy()
    assert (np.abs(sig[:k] - orc.Stilde[:k]) / orc.Stilde[:k]).max() < 1e-5


@pytest.mark.parametrize("m,n,k,l,i,lda,v_tol", [
    (1037, 334, 5, 7, 2, 336, 1e-4),      # ragged rows and K tails, padded lda
    (777, 200, 1, 1, 3, None, 1e-4),      # l = 1
    (900, 300, 6, 8, 0, None, 1e-4),      # i = 0
    (4000, 1500, 30, 40, 2, None, 2e-3),  # several Z tiles in the T pass (L = 120)
    (5000, 1200, 40, 70, 2, None, 2e-3),  # two forward column tiles (l = 70)
    (6100, 1002, 40, 60, 2, None, 2e-3),  # T pass over 180 columns in one read of A, ragged column tile
    (3000, 900, 20, 64, 1, None, 2e-3),   # T pass of exactly 128 columns; pass 0 adjoint of 65 (ones column)
    (2500, 640, 30, 48, 3, 644, 2e-3),    # T pass of exactly 192 columns, padded lda
])
def test_split_shapes_and_edges(m, n, k, l, i, lda, v_tol):
    sigma = 0.93 ** np.arange(n, dtype=np.float64)
    p = F.svd_problem(1000 + m, m, n, sigma)
    G = F.gaussian_G(1000 + m, n, l)
    orc = O.rpca(p["A"], k, l, i, G)
    g = run_gpu(p["A"], k, l, i, G=G, lda=lda, flags=_flag())
    compare(g, orc, k, v_tol=v_tol)
    r_g = O.residual_exact(p["A"], g[0], g[1], g[2])
    r_o = O.residual_exact(p["A"], orc.U, orc.S, orc.V)
    assert abs(r_g - r_o) / r_o < 1e-5


def test_split_centered_parity():
    """Low-rank + noise + U(0,1) column offsets, centred, including the pass-0 column sums."""
    m, n, r = 6000, 800, 12
    sig = 1.0 / np.arange(1, r + 1)
    p = F.lowrank_noise(31, m, n, r, sig, 1e-3, True)
    k, l, i = 10, 14, 2
    G = F.gaussian_G(31, n, l)
    orc = O.rpca(p["A"], k, l, i, G, center=True)
    g = run_gpu(p["A"], k, l, i, G=G, center=True, flags=_flag())
    compare(g, orc, k, n_vec=4)
    mu = g[3].state("MU").cpu().numpy()
    assert np.abs(mu - orc.mu).max() < 1e-9 * np.abs(p["A"]).max()
    assert np.abs(np.ones(m) @ g[0]).max() < 1e-4


def test_split_agrees_with_float32_kernels():
    """Same inputs through both kernel families: singular values agree to 1e-6 relative."""
    p = F.plain_small(seed=9, m=3000, n=900)
    k, l, i = 12, 16, 2
    G = F.gaussian_G(9, 900, l)
    a = run_gpu(p["A"], k, l, i, G=G)
    b = run_gpu(p["A"], k, l, i, G=G, flags=_flag())
    rel = np.abs(a[1] - b[1]) / a[1]
    print(f"  sigma float32 vs split max rel {rel.max():.3e}")
    assert rel.max() < 1e-6


def test_split_unsupported_cases():
    """Odd n and low-precision storage are rejected at planning."""
    _need_gpu()
    from paper_1007_5510_amd import rpca
    with pytest.raises(RuntimeError):
        rpca.Plan(100, 51, 2, 3, 1, flags=_flag())
    with pytest.raises(RuntimeError):
        rpca.Plan(100, 64, 2, 3, 1, storage="bf16", flags=_flag())


@pytest.mark.parametrize("split", [False, True])
def test_t_pass_elementwise_against_float64(split):
    """Step 3 on its own: T = (A - 1 mu^T)^T Q element by element against the float64 product
    with the device's own Q, each error scaled by (|A - 1 mu^T|^T |Q|), the bound of a rounded
    dot product.  180 columns in one read of A (float32: adj_wide_kernel, split: adj_x6w_kernel),
    centred, ragged last column tile.  Measured 2.4e-8 on both paths; the bar is 1e-6."""
    m, n, r = 6100, 1002, 12
    p = F.lowrank_noise(41, m, n, r, 1.0 / np.arange(1, r + 1), 1e-3, True)
    k, l, i = 40, 60, 2
    G = F.gaussian_G(41, n, l)
    g = run_gpu(p["A"], k, l, i, G=G, center=True, flags=_flag() if split else 0)
    Q = g[3].state("Q").cpu().numpy()
    T = g[3].state("T").cpu().numpy()
    A = np.asarray(p["A"], dtype=np.float32).astype(np.float64)  # the values the device holds
    Ac = A - A.mean(axis=0)
    Tref = Ac.T @ Q
    rel = np.abs(T - Tref) / (np.abs(Ac).T @ np.abs(Q))
    print(f"  T max error / dot-product bound {rel.max():.3e}")
    assert T.shape == (n, (i + 1) * l)
    assert rel.max() < 1e-6
