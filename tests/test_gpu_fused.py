"""Single-read power steps (panel_fused.hip): each power step of Step 1 reads the float32 A once
and produces the block H^(j) and the adjoint partial sums together (Section 4.1: every
contribution of a row made while the row is at hand).  Checked against the float64 oracle on the
same G, against the two-launch power steps on the same matrix, for ragged shapes and both group
layouts (one XCD per group for narrow A, two for wide A), and for bit-identical repeats."""
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


def _run(A, k, l, i, G, center=False, flags=None, lda=None):
    from paper_1007_5510_amd import rpca, _lib
    flags = _lib.FLAG_FUSED if flags is None else flags
    m, n = A.shape
    lda = lda or n
    buf = torch.zeros((m, lda), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    Gd = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda()
    p = rpca.Plan(m, n, k, l, i, center=center, flags=flags | _lib.FLAG_KEEP_STATE | _lib.FLAG_PROFILE)
    print(f"  factor m={m} n={n} k={k} l={l} i={i} center={center} lda={lda} flags={flags}", flush=True)
    U, S, V = p.factor(buf[:, :n], G=Gd)
    torch.cuda.synchronize()
    return U.cpu().double().numpy(), S.cpu().double().numpy(), V.cpu().double().numpy(), p


def _vector_bounds(A, orc, k, center):
    """Per-column bounds max(1e-4, 10 e_j), e_j the oracle's own change when its Step 1 blocks are
    rounded to float32 (the float32 path stores H in float32)."""
    reader = O.PanelReader(A, O.PANEL_ROWS, orc.mu if center else None)
    r = O.steps_2_to_6(reader, [h.astype(np.float32).astype(np.float64) for h in orc.H_blocks], k)
    eu = np.linalg.norm(r.U - orc.U, axis=0)
    ev = np.linalg.norm(r.V - orc.V, axis=0)
    return np.maximum(1e-4, 10.0 * eu), np.maximum(1e-4, 10.0 * ev)


def _check(g, orc, A, k, l, i, center):
    U, S, V, plan = g
    st = plan.stats()
    assert st["fused_launches"] == i, st          # the fused kernel ran every power step
    assert st["a_reads"] == i + 2                 # one read per pass of the schedule
    rel = np.abs(S - orc.S) / orc.S
    tu, tv = _vector_bounds(A, orc, k, center)
    eu = np.linalg.norm(U - orc.U, axis=0)
    ev = np.linalg.norm(V - orc.V, axis=0)
    print(f"  sigma rel err {rel.max():.3e}, U err {eu.max():.3e} (bound {tu[eu.argmax()]:.1e}), "
          f"V err {ev.max():.3e} (bound {tv[ev.argmax()]:.1e})")
    assert rel.max() <= 1e-5
    assert np.all(eu <= tu) and np.all(ev <= tv)
    # the blocks of Step 1 (up to the positive block scales) against the oracle's
    H = plan.state("H").cpu().double().numpy()
    scale = np.cumprod(plan.state("HSCALE").cpu().numpy())
    for j in range(i + 1):
        Hj = H[:, j * l:(j + 1) * l] / scale[j]
        err = np.linalg.norm(Hj - orc.H_blocks[j]) / np.linalg.norm(orc.H_blocks[j])
        print(f"  H^({j}) rel err {err:.3e}")
        assert err < 2e-6


@pytest.mark.parametrize("center", [False, True])
def test_fused_parity(center):
    """40000 x 1200 (one XCD per group), sigma_j = 0.9^(j-1), k = 20, l = 24, i = 2."""
    _need_gpu()
    m, n, k, l, i = 40000, 1200, 20, 24, 2
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    A = F.svd_problem(6200, m, n, sigma)["A"]
    if center:
        A = (A + F.column_offsets(6200, n).astype(np.float32)[None, :]).astype(np.float32)
    G = F.gaussian_G(6200, n, l)
    orc = O.rpca(A, k, l, i, G, center=center)
    g = _run(A, k, l, i, G, center=center)
    _check(g, orc, A, k, l, i, center)
    if center:
        mu = g[3].state("MU").cpu().numpy()
        assert np.abs(mu - A.astype(np.float64).mean(axis=0)).max() <= 1e-9 * np.abs(A).max()


def test_fused_ragged_scalar_loads():
    """m, n not multiples of 16 or of the group count, odd leading dimension (scalar loads), l + 1 = 8."""
    _need_gpu()
    m, n, k, l, i = 33333, 1037, 5, 7, 2
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    A = F.svd_problem(6300, m, n, sigma)["A"]
    A = (A + F.column_offsets(6300, n).astype(np.float32)[None, :]).astype(np.float32)
    G = F.gaussian_G(6300, n, l)
    orc = O.rpca(A, k, l, i, G, center=True)
    g = _run(A, k, l, i, G, center=True, lda=1041)
    _check(g, orc, A, k, l, i, True)


def test_fused_two_xcd_groups():
    """n = 10300 needs 21 column tiles per CU in one-XCD groups, so the groups span two XCDs (64 CUs,
    at most 20 tiles each); k = 10, l = 12, i = 1."""
    _need_gpu()
    m, n, k, l, i = 32768, 10300, 10, 12, 1
    sigma = 0.85 ** np.arange(n, dtype=np.float64)
    A = F.svd_problem(6400, m, n, sigma)["A"]
    G = F.gaussian_G(6400, n, l)
    orc = O.rpca(A, k, l, i, G)
    g = _run(A, k, l, i, G)
    _check(g, orc, A, k, l, i, False)


def test_fused_matches_two_launch_and_repeats_bitwise():
    """The same matrix with fused and with two-launch power steps: the blocks H agree to float32
    rounding and the singular values to 1e-6; two fused runs give identical bits (every sum is
    taken in a fixed order)."""
    _need_gpu()
    from paper_1007_5510_amd import _lib
    m, n, k, l, i = 36000, 2000, 12, 16, 2
    sigma = 0.92 ** np.arange(n, dtype=np.float64)
    A = F.svd_problem(6500, m, n, sigma)["A"]
    A = (A + F.column_offsets(6500, n).astype(np.float32)[None, :]).astype(np.float32)
    G = F.gaussian_G(6500, n, l)
    a = _run(A, k, l, i, G, center=True)
    b = _run(A, k, l, i, G, center=True, flags=0)
    c = _run(A, k, l, i, G, center=True)
    assert a[3].stats()["fused_launches"] == i and b[3].stats()["fused_launches"] == 0
    assert b[3].stats()["a_reads"] == 2 * i + 2 and a[3].stats()["a_reads"] == i + 2
    Ha = a[3].state("H").cpu().double().numpy()
    Hb = b[3].state("H").cpu().double().numpy()
    for j in range(i + 1):
        blk = slice(j * l, (j + 1) * l)
        err = np.linalg.norm(Ha[:, blk] - Hb[:, blk]) / np.linalg.norm(Hb[:, blk])
        print(f"  H^({j}) fused vs two-launch {err:.3e}")
        assert err < 2e-6
    assert np.abs(a[1] - b[1]).max() / b[1][0] < 1e-6
    for x, y in zip(a[:3], c[:3]):
        assert np.array_equal(x, y)
