"""GPU parity of the direct method (Algorithm DBS with window-sum
smoothing) against the FP64 oracle.

Every step is FP64 on both sides, so the bar is normwise:
max|B - B_oracle| <= 1e-10 max|B_oracle| over the principal domain (the
rounding of DFTs of length <= 65536 and of running sums over a few
thousand terms sits near 1e-14).  Whole grids are compared up to P = 300;
larger grids at sampled points, each evaluated by the oracle's explicit
box sum."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _hos():
    import paper_1805_11775_amd as hos
    assert hos.hos_device_check() == hos.HOS_OK, "no gfx950 device"
    return hos


def _run(x, P, M3, center=True, **kw):
    hos = _hos()
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    print("case: n=%d P=%d M3=%d dtype=%s center=%s %s" % (t.numel(), P, M3, t.dtype,
                                                           center, kw), flush=True)
    B = hos.dbs(t, P, M3, center=center, **kw)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def _err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n,P,M3,f32", [
    (64, 64, 5, False),       # one part, box wraps around the grid
    (300, 30, 4, True),       # ten parts, even box
    (97, 32, 1, False),       # no smoothing, trailing samples unused
    (40, 40, 40, False),      # box as wide as the grid
    (700, 300, 7, True),      # two parts, P = 2^2 3 5^2
    (4096, 256, 16, True),    # sixteen parts
    (1000, 250, 129, False),  # 512-wide strips
    (5, 2, 1, False), (6, 3, 2, True),   # the smallest grids
])
def test_whole_grid(n, P, M3, f32):
    x = synth.quadratic_process(n, 100 + n + M3)
    if f32:
        x = x.astype(np.float32)
    B = _run(x, P, M3)
    ref = oracle.dbs(x, P, M3)
    if np.max(np.abs(ref)) == 0.0:
        assert np.max(np.abs(B)) < 1e-12
        return
    e = _err(B, ref)
    print("rel err %.3e" % e)
    assert e < TOL


def _sampled(x, P, M3, B, count=48, seed=0):
    k1, k2 = oracle.pd_indices(P) if P <= 4096 else _pd_big(P)
    rng = np.random.default_rng(seed)
    pick = np.unique(np.concatenate([rng.integers(0, k1.size, count),
                                     [0, k1.size - 1, k1.size // 2]]))
    ref = oracle.dbs_at(x, P, M3, k1[pick], k2[pick])
    e = float(np.max(np.abs(B[pick] - ref)) / np.max(np.abs(ref)))
    print("sampled rel err %.3e over %d points" % (e, pick.size))
    return e


def _pd_big(P):
    """Principal-domain indices in the same order, vectorised per row."""
    H = (P - 1) // 2
    rows = np.arange(H + 1)
    lens = np.minimum(rows, H - rows) + 1
    k1 = np.repeat(rows, lens)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    k2 = np.arange(k1.size) - np.repeat(starts, lens)
    return k1, k2


@pytest.mark.parametrize("n,P,M3", [
    (2048 * 3, 2048, 300),     # 1024-wide strips, three parts
    (8192, 8192, 21),          # two-pass part DFT (64 x 128), one part
    (12000, 6000, 100),        # two-pass DFT with part sums (K = 2)
    (4096, 4096, 1500),        # 2048-wide strips, 549 output columns each
    (16384, 16384, 2048),      # the largest box: 2048-wide strips of one output column
])
def test_sampled_grids(n, P, M3):
    x = synth.iid_exp_centered(n, 7).astype(np.float32)
    B = _run(x, P, M3)
    assert B.size == len(_pd_big(P)[0])
    assert _sampled(x, P, M3, B) < TOL


def test_uncentred_constant_closed_form():
    """A constant c without mean removal: only F(0) = P c is nonzero, so
    the raw bispectrum is P^2 c^3 at the origin alone and the smoothed value
    is that over M3^2 wherever the box covers the origin (k1, k2 <= lo here,
    with the wrap-around from the top rows); with the mean removed, zero."""
    P, M3, c = 64, 5, 1.5
    x = np.full(3 * P, c)
    B = _run(x, P, M3, center=False)
    k1, k2 = oracle.pd_indices(P)
    lo, hi = M3 // 2, M3 - 1 - M3 // 2
    H = (P - 1) // 2
    cover = lambda k: (k <= lo) | (k >= P - hi)
    expect = np.where(cover(k1) & cover(k2), P * P * c ** 3 / M3 ** 2, 0.0)
    assert k1.max() == H
    assert np.max(np.abs(B - expect)) < 1e-12 * P * P * c ** 3
    assert np.max(np.abs(_run(x, P, M3))) < 1e-9


def test_workload_sampled():
    """n = 2^16 float32 quadratic process, one part, 1023-wide box (the
    benchmark shape and launch configuration): sampled points against the
    oracle's box sums."""
    x, cfg = synth.workload_dbs()
    B = _run(x, cfg["P"], cfg["M3"])
    assert _sampled(x, cfg["P"], cfg["M3"], B, count=40) < TOL


def test_deterministic_workspace_independent_and_row_runs():
    hos = _hos()
    x = torch.from_numpy(synth.quadratic_process(30000, 4).astype(np.float32)).cuda()
    P, M3 = 3000, 200
    Ba = hos.dbs(x, P, M3)
    nb = hos.hos_dbs_workspace(x.numel(), P, M3)
    ws = torch.full((nb,), 0xFF, dtype=torch.uint8, device="cuda")   # NaN bytes
    Bb = hos.dbs(x, P, M3, workspace=ws)
    Bc = hos.dbs(x, P, M3, seg_rows=37)
    torch.cuda.synchronize()
    assert torch.equal(Ba, Bb) and not torch.isnan(Ba).any()
    a, c = Ba.cpu().numpy(), Bc.cpu().numpy()
    assert np.max(np.abs(a - c)) < 1e-12 * np.max(np.abs(a))
    x1 = torch.from_numpy(synth.quadratic_process(65536, 5).astype(np.float32)).cuda()
    B1 = hos.dbs(x1, 65536, 255)
    B2 = hos.dbs(x1, 65536, 255, seg_rows=300)
    torch.cuda.synchronize()
    d = (B1 - B2).abs().max().item() / B1.abs().max().item()
    print("row-run split difference %.3e" % d)
    assert d < 1e-12
