"""m < n: Section 3 takes n <= m and applies the method to A^T otherwise.

The library plans the problem of B = A~^T (n x m) and runs its Steps 1 and 3 on the stored A with
the roles of the products exchanged (B X = A~^T X as an adjoint launch, B^T Y = A~ Y as a forward
launch); U and V of A are V and U of B.  The oracle does the same by transposing A (after centring
its columns) and exchanging the outputs, so both sides share G (m x l, the test matrix of A^T's
problem) and the sign rule (applied to the right singular vectors of A^T, i.e. to u_j).
"""
import numpy as np
import pytest

from synth import fixtures as F
from oracle import rpca_oracle as O
from tests.test_gpu_parity import _need_gpu, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run_wide(A, k, l, i, G=None, center=False, lda=None, seed=0, flags=0):
    _need_gpu()
    from paper_1007_5510_amd import rpca, _lib
    m, n = A.shape
    lda = lda or n
    buf = torch.zeros((m, lda), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    Gd = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda() if G is not None else None
    p = rpca.Plan(m, n, k, l, i, center=center, seed=seed, flags=flags | _lib.FLAG_PROFILE)
    U, S, V = p.factor(buf[:, :n], G=Gd)
    torch.cuda.synchronize()
    assert U.shape == (m, k) and V.shape == (n, k)
    return U.cpu().double().numpy(), S.cpu().double().numpy(), V.cpu().double().numpy(), p


def test_wide_plain_parity():
    """The plain small matrix transposed: 1000 x 2000, sigma_j = 0.9^(j-1), k = 10, l = 12, i = 1."""
    p = F.plain_small()
    A = np.ascontiguousarray(p["A"].T)
    k, l, i = p["k"], p["l"], p["i"]
    G = F.gaussian_G(1007, 1000, l)
    orc = O.rpca(A, k, l, i, G)
    g = run_wide(A, k, l, i, G=G)
    compare(g, orc, k)
    res = O.residual_exact(A, g[0], g[1], g[2])
    print(f"  residual / sigma_(k+1) {res / 0.9 ** 10:.5f}")
    assert res / 0.9 ** 10 <= 1.1
    st = g[3].stats()
    assert st["passes"] == i + 2 and st["a_reads"] == 2 * i + 2 and st["qr_fallback"] == 0


@pytest.mark.parametrize("m,n,k,l,i,lda", [
    (333, 1037, 5, 7, 2, None),   # ragged, lda % 4 != 0
    (333, 1037, 5, 7, 2, 1040),   # padded lda (vector loads)
    (300, 900, 6, 8, 0, None),    # i = 0
    (1500, 4000, 30, 40, 2, None),  # L = 120: several Z tiles in the forward launch of Step 3
])
def test_wide_shapes(m, n, k, l, i, lda):
    sigma = 0.93 ** np.arange(m, dtype=np.float64)
    p = F.svd_problem(2000 + m, n, m, sigma)          # n x m, transposed below
    A = np.ascontiguousarray(p["A"].T)
    G = F.gaussian_G(2000 + m, m, l)
    orc = O.rpca(A, k, l, i, G)
    g = run_wide(A, k, l, i, G=G, lda=lda)
    compare(g, orc, k, v_tol=1e-4 if (i + 1) * l < 100 else 2e-3)
    r_g = O.residual_exact(A, g[0], g[1], g[2])
    r_o = O.residual_exact(A, orc.U, orc.S, orc.V)
    print(f"  residual gpu {r_g:.6e} oracle {r_o:.6e}")
    assert abs(r_g - r_o) / r_o < 1e-5


def test_wide_centered_parity():
    """Low-rank + noise with column offsets, 800 x 6000, centred (column means of A removed)."""
    m, n, r = 6000, 800, 12
    p = F.lowrank_noise(41, m, n, r, 1.0 / np.arange(1, r + 1), 1e-3, False)
    A = np.ascontiguousarray(p["A"].T)                 # 800 x 6000
    A = (A + F.column_offsets(41, 6000)[None, :].astype(np.float32)).astype(np.float32)
    k, l, i = 10, 14, 2
    G = F.gaussian_G(41, 800, l)
    orc = O.rpca(A, k, l, i, G, center=True)
    g = run_wide(A, k, l, i, G=G, center=True)
    compare(g, orc, k, n_vec=4)
    # U spans directions of range(A~), which is orthogonal to 1
    assert np.abs(np.ones(800) @ g[0]).max() < 1e-4
    st = g[3].stats()
    assert st["passes"] == i + 3 and st["a_reads"] == 2 * i + 3  # plus the column-mean pass


def test_wide_generated_G():
    """G drawn from the seed for A^T's problem equals the generator's m x l matrix."""
    p = F.plain_small(seed=6, m=1300, n=500)
    A = np.ascontiguousarray(p["A"].T)                 # 500 x 1300
    k, l, i, seed = 6, 8, 1, 97531
    G = F.gaussian_G(seed, 500, l)
    orc = O.rpca(A, k, l, i, G)
    g = run_wide(A, k, l, i, G=None, seed=seed)
    compare(g, orc, k)


def test_wide_refusals():
    from paper_1007_5510_amd import rpca, _lib
    _need_gpu()
    for flags in (_lib.FLAG_KEEP_STATE, _lib.FLAG_SPLIT_BF16, _lib.FLAG_FP64_STEP1):
        with pytest.raises(_lib.RPCAError) as e:
            rpca.Plan(200, 500, 5, 6, 1, flags=flags)
        assert e.value.code == 2
    with pytest.raises(_lib.RPCAError) as e:
        rpca.Plan(200, 500, 5, 6, 1, storage="bf16")
    assert e.value.code == 2
    with pytest.raises(_lib.RPCAError) as e:
        rpca.Plan(30, 500, 10, 12, 1)                  # (i+1) l = 24 > min(m, n) - k = 20
    assert e.value.code == 1
    A = torch.zeros((200, 500), dtype=torch.float32, device="cuda")
    with rpca.Plan(200, 500, 5, 6, 1) as p:
        with pytest.raises(ValueError):
            p.factor(A, G=torch.zeros((500, 6), dtype=torch.float32, device="cuda"))  # G must be 200 x 6
