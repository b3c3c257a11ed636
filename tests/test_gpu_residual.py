"""rpca_residual: the Appendix estimator p_{j,q}(D) of ||D||_2, D = A~ - U S V^T, on the GPU against
the oracle's estimator with the same start vectors (Philox stream 9) and against the exact norm."""
import os

import numpy as np
import pytest

from synth import fixtures as F
from synth import philox as PX
from oracle import rpca_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIBDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_5510_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(os.path.join(LIBDIR, "librpca.so")):
        pytest.fail("librpca.so is not built (the GPU path has no fallback)")


@pytest.mark.parametrize("center,j,q", [(False, 6, 10), (True, 6, 10), (False, 3, 4), (False, 1, 1)])
def test_residual_estimate_matches_oracle(center, j, q):
    _need_gpu()
    from paper_1007_5510_amd import rpca
    m, n, k, l, i = 4000, 900, 10, 12, 1
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    A = F.svd_problem(6100, m, n, sigma)["A"]
    if center:
        A = (A + F.column_offsets(6100, n).astype(np.float32)[None, :]).astype(np.float32)
    G = F.gaussian_G(6100, n, l)
    seed = 6101
    p = rpca.Plan(m, n, k, l, i, center=center)
    Ad = torch.from_numpy(A).cuda()
    U, S, V = p.factor(Ad, G=torch.from_numpy(G.astype(np.float32)).cuda())
    est = p.residual(Ad, U, S, V, j=j, q=q, seed=seed)
    Uh, Sh, Vh = (t.cpu().double().numpy() for t in (U, S, V))
    starts = PX.normal_matrix(seed, 9, n, q)
    ref = O.residual_estimate(A, Uh, Sh, Vh, starts, center=center, j=j)
    exact = O.residual_exact(A, Uh, Sh, Vh, center=center)
    print(f"  center={center} j={j} q={q}: gpu {est:.8f} oracle {ref:.8f} exact {exact:.8f}")
    assert abs(est - ref) <= 1e-5 * ref
    assert est <= exact * (1 + 1e-6)
    if j == 6:
        assert est >= 0.5 * exact  # fails with probability below the Appendix bound


def test_residual_rejects_bad_arguments():
    _need_gpu()
    from paper_1007_5510_amd import rpca, _lib
    m, n = 600, 200
    p = rpca.Plan(m, n, 4, 6, 1)
    A = torch.randn(m, n, device="cuda")
    U, S, V = p.factor(A)
    with pytest.raises(_lib.RPCAError):
        p.residual(A, U, S, V, j=0)
