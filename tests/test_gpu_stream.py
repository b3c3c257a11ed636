"""Streamed sources (Section 4): A in pinned host memory or produced by a callback, moved to the
GPU in row panels, one host-link transfer per pass, or generated on the device panel by panel in
every pass (Section 4.1), against the oracle and the in-core path."""
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


def _f32_block_tolerances(A, orc, k, center=False):
    """Per-column vector bounds max(1e-4, 10 e_j): e_j is how far the oracle's own u_j (v_j) moves
    when its Step 1 blocks are rounded to float32 and Steps 2-6 are redone in float64."""
    reader = O.PanelReader(A, O.PANEL_ROWS, orc.mu if center else None)
    r = O.steps_2_to_6(reader, [h.astype(np.float32).astype(np.float64) for h in orc.H_blocks], k)
    eu = np.linalg.norm(r.U - orc.U, axis=0)
    ev = np.linalg.norm(r.V - orc.V, axis=0)
    return np.maximum(1e-4, 10.0 * eu), np.maximum(1e-4, 10.0 * ev)


def _problem(seed, m, n, center):
    sigma = 0.9 ** np.arange(min(n, 300), dtype=np.float64)
    A = F.svd_problem(seed, m, n, sigma)["A"]
    if center:
        A = (A + F.column_offsets(seed, n).astype(np.float32)[None, :]).astype(np.float32)
    return A


def _pinned(A, ld=None):
    m, n = A.shape
    ld = ld or n
    buf = torch.zeros((m, ld), dtype=torch.float32, pin_memory=True)
    buf[:, :n] = torch.from_numpy(A)
    return buf[:, :n]


def _run(A, k, l, i, G, center, source, panel_rows, ld=None):
    from paper_1007_5510_amd import rpca, _lib
    m, n = A.shape
    p = rpca.Plan(m, n, k, l, i, center=center, source=source, panel_rows=panel_rows, flags=_lib.FLAG_PROFILE)
    Gd = torch.from_numpy(G.astype(np.float32)).cuda()
    if source == "host_pinned":
        U, S, V = p.factor(_pinned(A, ld), G=Gd)
    elif source == "callback":
        def fill(row0, nrows, buf):
            buf[:, :n] = A[row0:row0 + nrows]
        U, S, V = p.factor(None, G=Gd, panel_fn=fill)
    elif source == "device_callback":
        from synth import gpu as SG
        Ad = torch.from_numpy(A).cuda()
        torch.cuda.synchronize()

        def fill_dev(row0, nrows, dst, ld, stream):
            SG.copy_rows_at(dst, ld, Ad, row0, nrows, stream)
        U, S, V = p.factor(None, G=Gd, panel_fn=fill_dev)
    else:
        U, S, V = p.factor(torch.from_numpy(A).cuda(), G=Gd)
    torch.cuda.synchronize()
    return U.cpu().double().numpy(), S.cpu().double().numpy(), V.cpu().double().numpy(), p.stats()


@pytest.mark.parametrize("source,center,panel_rows,ld", [
    ("host_pinned", False, 8192, None),    # 7 panels, ragged last panel (50000 = 6 * 8192 + 848)
    ("host_pinned", True, 8192, None),
    ("host_pinned", False, 4096, 1040),    # lda > n: pitched copies
    ("callback", False, 8192, None),
    ("callback", True, 16384, None),
    ("device_callback", False, 8192, None),
    ("device_callback", True, 16384, None),
])
def test_streamed_parity(source, center, panel_rows, ld):
    _need_gpu()
    m, n, k, l, i = 50000, 1000, 10, 12, 2
    A = _problem(4000, m, n, center)
    G = F.gaussian_G(4000, n, l)
    orc = O.rpca(A, k, l, i, G, center=center)
    U, S, V, st = _run(A, k, l, i, G, center, source, panel_rows, ld)
    rel = np.abs(S - orc.S) / orc.S
    du = np.linalg.norm(U - orc.U, axis=0).max()
    dv = np.linalg.norm(V - orc.V, axis=0).max()
    print(f"  {source} center={center} panels of {panel_rows}: sigma {rel.max():.2e} U {du:.2e} V {dv:.2e} "
          f"passes {st['passes']} h2d {st['h2d_bytes'] / 1e9:.2f} GB")
    assert rel.max() < 1e-5
    assert du < 1e-4 and dv < 1e-4
    passes = i + 2 + (1 if center else 0)
    assert st["passes"] == passes
    assert st["h2d_bytes"] == (0 if source == "device_callback" else passes * m * n * 4)


def test_streamed_matches_in_core():
    """Same inputs through the device and the host-pinned source: the same factorisation."""
    _need_gpu()
    m, n, k, l, i = 30000, 700, 8, 10, 1
    A = _problem(4100, m, n, False)
    G = F.gaussian_G(4100, n, l)
    a = _run(A, k, l, i, G, False, "device", 0)
    b = _run(A, k, l, i, G, False, "host_pinned", 7000)
    assert np.abs(a[1] - b[1]).max() / a[1][0] < 1e-6
    assert np.linalg.norm(a[2] - b[2], axis=0).max() < 1e-5


def test_callback_error_is_reported():
    _need_gpu()
    from paper_1007_5510_amd import rpca, _lib
    m, n = 20000, 300
    p = rpca.Plan(m, n, 4, 6, 1, source="callback", panel_rows=4096)

    def fill(row0, nrows, buf):
        if row0 >= 8192:
            raise RuntimeError("data source failed")
        buf[:, :n] = 1.0
    with pytest.raises(_lib.RPCAError) as e:
        p.factor(None, panel_fn=fill)
    assert e.value.code == 5  # RPCA_ERR_CALLBACK


def test_device_callback_matches_host_pinned():
    """Rows generated on the device and rows copied from pinned host memory go through the same
    panel kernels with the same panel boundaries: the results are identical."""
    _need_gpu()
    m, n, k, l, i = 30000, 700, 8, 10, 2
    A = _problem(4200, m, n, False)
    G = F.gaussian_G(4200, n, l)
    a = _run(A, k, l, i, G, False, "host_pinned", 5000)
    b = _run(A, k, l, i, G, False, "device_callback", 5000)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert b[3]["h2d_bytes"] == 0 and b[3]["passes"] == a[3]["passes"]


def test_device_regenerated_rows_match_in_core():
    """Rows regenerated by the seeded device generator in every pass (the on-the-fly mode) and the
    same matrix generated once and factored in core, each against the float64 oracle run on that
    matrix with the same G: singular values within 1e-5 relative (the float32 target).  Singular
    vectors: the float32 path keeps the Step 1 blocks H in float32, so its vectors cannot be closer
    to the oracle's than the oracle's own vectors move when its H is rounded to float32; with
    sigma_j = exp(-j/10) and i = 2 the last wanted columns of H^(2) carry (sigma_20/sigma_1)^5 ~ 1e-4
    of the block's norm, and that rounding alone moves u_20 by ~4e-4.  Each column j is therefore
    held to max(1e-4, 10 e_j), e_j the oracle's change under that rounding (the factor 10 covers
    float32 accumulation in the products against a single rounding of the stored block).  The two
    device runs split the row sums differently (6000-row panels against the in-core row split);
    their singular values also agree with each other to 1e-6 relative."""
    _need_gpu()
    from synth import gpu as SG
    from paper_1007_5510_amd import rpca, _lib
    m, n, r, k, l, i, seed = 40000, 1200, 30, 20, 24, 2, 4300
    Ur, Vr = F.lowrank_factors(seed, m, n, r)
    sig = np.exp(-np.arange(1, r + 1, dtype=np.float64) / 10.0)
    Ur_d = torch.from_numpy(np.ascontiguousarray(Ur)).cuda()
    Vr_d = torch.from_numpy(np.ascontiguousarray(Vr)).cuda()
    s_d = torch.from_numpy(sig).cuda()
    A = torch.empty((m, n), dtype=torch.float32, device="cuda")
    SG.lowrank_noise_into(A, 0, Ur_d, s_d, Vr_d, 1e-4, None, seed)
    torch.cuda.synchronize()
    Gh = F.gaussian_G(seed, n, l).astype(np.float32)
    G = torch.from_numpy(Gh).cuda()
    p0 = rpca.Plan(m, n, k, l, i)
    U0, S0, V0 = p0.factor(A, G=G)
    calls = []

    def gen(row0, nrows, dst, ld, stream):
        calls.append(row0)
        SG.lowrank_noise_at(dst, ld, nrows, n, row0, Ur_d, s_d, Vr_d, 1e-4, None, seed, stream)
    p1 = rpca.Plan(m, n, k, l, i, source="device_callback", panel_rows=6000, flags=_lib.FLAG_PROFILE)
    U1, S1, V1 = p1.factor(None, G=G, panel_fn=gen)
    torch.cuda.synchronize()
    assert len(calls) == (i + 2) * ((m + 5999) // 6000)  # every pass regenerates every panel
    Ah = A.cpu().numpy()
    orc = O.rpca(Ah, k, l, i, Gh)
    tol_u, tol_v = _f32_block_tolerances(Ah, orc, k)
    for name, (U_, S_, V_) in (("in core", (U0, S0, V0)), ("regenerated", (U1, S1, V1))):
        S_ = S_.cpu().double().numpy()
        U_, V_ = U_.cpu().double().numpy(), V_.cpu().double().numpy()
        es = (np.abs(S_ - orc.S) / orc.S).max()
        eu = np.linalg.norm(U_ - orc.U, axis=0)
        ev = np.linalg.norm(V_ - orc.V, axis=0)
        print(f"  {name}: sigma rel err {es:.2e}, U err {eu.max():.2e} (col {eu.argmax()}, bound "
              f"{tol_u[eu.argmax()]:.2e}), V err {ev.max():.2e} (bound {tol_v[ev.argmax()]:.2e})")
        assert es <= 1e-5 and np.all(eu <= tol_u) and np.all(ev <= tol_v)
    S0, S1 = S0.cpu().double().numpy(), S1.cpu().double().numpy()
    assert np.abs(S0 - S1).max() / S0[0] < 1e-6


def test_device_callback_error_is_reported():
    _need_gpu()
    from synth import gpu as SG
    from paper_1007_5510_amd import rpca, _lib
    m, n = 20000, 300
    Ad = torch.ones((m, n), dtype=torch.float32, device="cuda")
    p = rpca.Plan(m, n, 4, 6, 1, source="device_callback", panel_rows=4096)

    def fill(row0, nrows, dst, ld, stream):
        if row0 >= 8192:
            raise RuntimeError("generator failed")
        SG.copy_rows_at(dst, ld, Ad, row0, nrows, stream)
    with pytest.raises(_lib.RPCAError) as e:
        p.factor(None, panel_fn=fill)
    assert e.value.code == 5  # RPCA_ERR_CALLBACK
    torch.cuda.synchronize()
