"""The in-core float32 workload at its full size (200000 x 20000 low-rank + noise with column
offsets, k = 50, l = 60, i = 2, centred), in the launch configuration the benchmark times.

The float64 reference at this size is computed from A itself, streamed once to the host in row
chunks: the exact column means, sampled rows of the first block H^(0) = A~ G (Step 1, eq.
first_prod) one row at a time, and A~^T U.  Checked against them:

* the column means (pass 0's implicit ones column) within 1e-9 max|A|;
* sampled rows of H^(0) within 2e-6 relative (the float32 product bound used for the H blocks
  at the parity sizes);
* the identity A~^T U_k = V_k S_k, which the algorithm satisfies exactly for its computed T
  (T = A~^T Q, T = V~ S~ W^T and U = Q W give A~^T U = V~ S~), within the float32 accuracy
  target applied to the factorisation, 1e-5 ||S_k||_F (the worst-case size of a float32
  accumulation error of T, sqrt(m) u ||A~||_F sqrt(k) with u = 2^-24, is printed beside it);
* U and V orthonormal to 1e-5.
"""
import math

import numpy as np
import pytest

from synth import fixtures as F
from tests.test_gpu_parity import _need_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M, N, R, K, L, I, SEED = 200000, 20000, 50, 50, 60, 2, 0


def _workload():
    from synth import gpu as SG
    Ur, Vr = F.lowrank_factors(SEED, M, N, R)
    sigma = 1.0 / np.arange(1, R + 1, dtype=np.float64)
    off = F.column_offsets(SEED, N)
    A = torch.empty((M, N), dtype=torch.float32, device="cuda")
    SG.lowrank_noise_into(A, 0, torch.from_numpy(np.ascontiguousarray(Ur)).cuda(),
                          torch.from_numpy(sigma).cuda(), torch.from_numpy(np.ascontiguousarray(Vr)).cuda(),
                          1e-3, torch.from_numpy(off).cuda(), SEED)
    torch.cuda.synchronize()
    return A


def test_incore_full_size_sampled_and_invariants():
    _need_gpu()
    from paper_1007_5510_amd import rpca, _lib
    A = _workload()
    Gh = F.gaussian_G(SEED, N, L).astype(np.float32)
    plan = rpca.Plan(M, N, K, L, I, center=True, flags=_lib.FLAG_PROFILE)
    U, S, V = plan.factor(A, G=torch.from_numpy(Gh).cuda())
    torch.cuda.synchronize()
    st = plan.stats()
    print(f"  factor {st['ms_total']:.1f} ms, passes {st['passes']}, Step 2 level {st['qr_fallback']}")
    assert st["passes"] == I + 2
    U = U.cpu().double().numpy()
    S = S.cpu().double().numpy()
    V = V.cpu().double().numpy()
    H0 = plan.state("H").cpu().double().numpy()[:, :L]
    scale0 = float(plan.state("HSCALE").cpu().numpy()[0])
    mu_gpu = plan.state("MU").cpu().numpy()

    rows = np.unique(np.concatenate([np.array([0, 1, 127, 128, 4095, 4096, M - 2, M - 1]),
                                     np.random.default_rng(5).integers(0, M, 56)]))
    colsum = np.zeros(N)
    sqsum = np.zeros(N)
    AtU = np.zeros((N, K))
    Arows = {}
    chunk = 8192
    for r0 in range(0, M, chunk):
        r1 = min(M, r0 + chunk)
        Ac = A[r0:r1].cpu().numpy().astype(np.float64)
        colsum += Ac.sum(axis=0)
        sqsum += np.einsum("ij,ij->j", Ac, Ac)
        AtU += Ac.T @ U[r0:r1]
        for r in rows[(rows >= r0) & (rows < r1)]:
            Arows[int(r)] = Ac[r - r0].copy()
        del Ac
    mu = colsum / M
    lo, hi = torch.aminmax(A)
    amax = max(abs(float(lo.item())), abs(float(hi.item())))

    # column means of pass 0
    dmu = np.abs(mu_gpu - mu).max()
    print(f"  column means: max |mu_gpu - mu| {dmu:.2e} (max|A| {amax:.2f})")
    assert dmu <= 1e-9 * amax

    # sampled rows of H^(0) = (A - 1 mu^T) G, one row at a time
    errs = []
    for r in rows:
        ref = (Arows[int(r)] - mu) @ Gh.astype(np.float64)
        got = H0[r] / scale0
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"  sampled H^(0) rows: max rel err {max(errs):.2e} over {len(rows)} rows")
    assert max(errs) <= 2e-6

    # A~^T U_k = V_k S_k (exact for the computed T, up to its float32 accumulation)
    AtU_c = AtU - np.outer(mu, U.sum(axis=0))
    fro_At = math.sqrt(float((sqsum - M * mu * mu).sum()))
    resid = np.linalg.norm(AtU_c - V * S)
    bound = math.sqrt(M) * 2.0 ** -24 * fro_At * math.sqrt(K)
    print(f"  ||A~^T U - V S||_F {resid:.3e}, bound {bound:.3e} (||A~||_F {fro_At:.2f}, ||S||_F "
          f"{np.linalg.norm(S):.3f})")
    assert resid <= 1e-5 * np.linalg.norm(S)

    assert np.abs(U.T @ U - np.eye(K)).max() < 1e-5
    assert np.abs(V.T @ V - np.eye(K)).max() < 1e-5
    assert np.all(np.diff(S) <= 1e-6 * S[0])

