"""GPU parity of segment averaging (Algorithm DBS's split into parts, per-part mean removal and
average over parts, around the cumulant) against the FP64 oracle.  Bars as for one series: normwise
1e-6 (FP32 path) and 1e-5 (split paths) for c3 over the hexagon and for B
over the grid."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-6, "split_fp16": 1e-5, "split_bf16": 1e-5}


def _hos():
    import paper_1805_11775_amd as hos
    assert hos.hos_device_check() == hos.HOS_OK, "no gfx950 device"
    return hos


def _run(x, P, M, **kw):
    hos = _hos()
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    print("case: n=%d P=%d M=%d %s dtype=%s" % (t.numel(), P, M, kw, t.dtype), flush=True)
    c3, B = hos.bispectrum_segments(t, P, M, **kw)
    torch.cuda.synchronize()
    return c3.cpu().numpy(), B.cpu().numpy()


def _err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("path", list(TOL))
@pytest.mark.parametrize("n,P,M,window", [
    (4000, 1000, 20, "parzen"),     # four segments
    (5003, 1000, 33, "parzen"),     # trailing samples unused
    (3000, 3000, 64, "parzen"),     # one segment
    (9000, 300, 5, "parzen"),       # thirty short segments
    (2400, 600, 100, "parzen"),     # 4 x 4-block tiles
])
def test_parity(path, n, P, M, window):
    x = synth.quadratic_process(n, 40 + M).astype(np.float32)
    c3, B = _run(x, P, M, window=window, path=path)
    N = _hos().default_nfft(M, window)
    c_ref, B_ref = oracle.bispectrum_segments(x, P, M, N, window=window)
    e1, e2 = _err(c3, c_ref), _err(B, B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


def test_segment_means_removed():
    """A different constant added to every segment leaves the estimate
    unchanged up to rounding (each segment is centred on its own mean)."""
    P, K = 2000, 6
    x = synth.iid_exp_centered(P * K, 5)
    y = x + np.repeat(np.arange(K) * 3.0 - 5.0, P)
    c3x, Bx = _run(x, P, 24, path="fp32")
    c3y, By = _run(y, P, 24, path="fp32")
    assert _err(c3y, c3x) < 1e-6 and _err(By, Bx) < 1e-6


def test_float64_matches_plain_bispectrum_for_one_segment():
    hos = _hos()
    x = synth.cubic_process(5000, 3)
    t = torch.from_numpy(x).cuda()
    c3s, Bs = hos.bispectrum_segments(t, 5000, 40, path="fp32")
    c3p, Bp = hos.bispectrum(t, 40, path="fp32")
    torch.cuda.synchronize()
    assert _err(c3s.cpu().numpy(), c3p.cpu().numpy()) < 1e-6
    assert _err(Bs.cpu().numpy(), Bp.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_workload_sampled(path):
    """n = 2^20 float32 quadratic process in 16 segments of 65536, M = 512:
    sampled lags against the oracle's per-segment sums, averaged."""
    x, cfg = synth.workload_segments()
    P, M = cfg["P"], cfg["M"]
    c3, B = _run(x, P, M, path=path)
    rng = np.random.default_rng(8)
    w = rng.integers(-M, M + 1, (150, 2))
    w = w[np.abs(w[:, 0] - w[:, 1]) <= M]
    K = x.size // P
    ref = np.mean([oracle.c3_at(x[i * P:(i + 1) * P], w[:, 0], w[:, 1]) for i in range(K)], 0)
    e = float(np.max(np.abs(c3[w[:, 0] + M, w[:, 1] + M] - ref)) / np.max(np.abs(ref)))
    print("sampled rel err %.3e" % e)
    assert e < TOL[path]
    assert np.isfinite(B).all()
