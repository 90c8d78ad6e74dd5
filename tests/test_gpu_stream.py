"""GPU parity of the streamed bispectrum (a record in host memory, read in
pieces with an M-sample halo through a device workspace independent of n)
against the FP64 oracle, and against the in-memory call on the same record.
Bars as for one series (normwise 1e-6 FP32, 1e-5 split)."""
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


def _err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.mark.parametrize("path", list(TOL))
@pytest.mark.parametrize("n,M,piece", [
    (20000, 64, 4096),         # five pieces, the last one partial
    (8242, 100, 4096),         # last piece of 50 samples, shorter than M
    (5000, 33, 8192),          # one piece
    (8193, 20, 4096),          # last piece of one sample
])
def test_parity(path, n, M, piece):
    hos = _hos()
    x = synth.quadratic_process(n, 500 + n).astype(np.float32)
    print("case: n=%d M=%d piece=%d path=%s" % (n, M, piece, path), flush=True)
    c3, B = hos.bispectrum_streamed(torch.from_numpy(x), M, piece=piece, path=path)
    torch.cuda.synchronize()
    N = hos.default_nfft(M)
    c_ref, B_ref = oracle.bispectrum(x, M, N)
    e1, e2 = _err(c3.cpu().numpy(), c_ref), _err(B.cpu().numpy(), B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


def test_float64_pinned_and_uncentred():
    hos = _hos()
    x = synth.iid_exp_centered(12345, 7) + 3.0
    xt = torch.from_numpy(x).pin_memory()
    for center in (True, False):
        c3, B = hos.bispectrum_streamed(xt, 40, piece=4096, path="fp32", center=center)
        torch.cuda.synchronize()
        c_ref, B_ref = oracle.bispectrum(x, 40, hos.default_nfft(40), centered=center)
        assert _err(c3.cpu().numpy(), c_ref) < 1e-6 and _err(B.cpu().numpy(), B_ref) < 1e-6


@pytest.mark.parametrize("n,piece", [(20000, 4096), (5000, 8192)])
def test_pinned_read_in_place(n, piece):
    """A record in pinned memory is read in place by the first pass (a view
    at an offset into a larger pinned block; five pieces, and one piece);
    the result equals the pageable copy path's up to the order of the FP64
    additions of the mean, and the oracle's."""
    hos = _hos()
    x = synth.quadratic_process(n, 900 + n).astype(np.float32)
    blk = torch.zeros(n + 11, dtype=torch.float32).pin_memory()
    blk[5:5 + n] = torch.from_numpy(x)
    view = blk[5:5 + n]
    assert view.is_pinned() and view.data_ptr() != blk.data_ptr()
    print("case: pinned view n=%d piece=%d" % (n, piece), flush=True)
    cp, Bp = hos.bispectrum_streamed(view, 64, piece=piece, path="split_fp16")
    cq, Bq = hos.bispectrum_streamed(torch.from_numpy(x.copy()), 64, piece=piece,
                                     path="split_fp16")
    torch.cuda.synchronize()
    d1 = _err(cp.cpu().numpy(), cq.cpu().numpy())
    d2 = _err(Bp.cpu().numpy(), Bq.cpu().numpy())
    print("pinned vs pageable: c3 %.3e B %.3e" % (d1, d2))
    assert d1 < 1e-12 and d2 < 1e-12
    c_ref, B_ref = oracle.bispectrum(x, 64, hos.default_nfft(64))
    assert _err(cp.cpu().numpy(), c_ref) < TOL["split_fp16"]
    assert _err(Bp.cpu().numpy(), B_ref) < TOL["split_fp16"]


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_matches_in_memory_call_at_size(path):
    """n = 2^22 float32 quadratic process, M = 512, pieces of 2^20: the
    streamed result against the in-memory call on the same record (same
    operand rounding, same 512-sample accumulation blocks) and against the
    oracle at sampled lags."""
    hos = _hos()
    x = synth.quadratic_process(1 << 22, 77).astype(np.float32)
    xh = torch.from_numpy(x).pin_memory()   # held until the copies have landed
    cs, Bs = hos.bispectrum_streamed(xh, 512, piece=1 << 20, path=path)
    cm, Bm = hos.bispectrum(torch.from_numpy(x).cuda(), 512, path=path)
    torch.cuda.synchronize()
    cs, cm = cs.cpu().numpy(), cm.cpu().numpy()
    d1 = _err(cs, cm)
    d2 = _err(Bs.cpu().numpy(), Bm.cpu().numpy())
    print("streamed vs in-memory: c3 %.3e B %.3e" % (d1, d2))
    assert d1 < 1e-9 and d2 < 1e-9
    rng = np.random.default_rng(2)
    w = rng.integers(-512, 513, (120, 2))
    w = w[np.abs(w[:, 0] - w[:, 1]) <= 512]
    ref = oracle.c3_at(x, w[:, 0], w[:, 1])
    e = float(np.max(np.abs(cs[w[:, 0] + 512, w[:, 1] + 512] - ref)) / np.max(np.abs(ref)))
    print("sampled rel err %.3e" % e)
    assert e < TOL[path]


@pytest.mark.parametrize("path", list(TOL))
@pytest.mark.parametrize("n,M,piece,window", [
    (20000, 64, 4096, "parzen"),       # five pieces, halo 2M = 128
    (8242, 100, 4096, "parzen"),       # last piece of 50 samples, halo 200
    (13000, 150, 4096, "separable"),   # corners weighted by the window
    (9000, 30, 4096, "none"),
])
def test_full_square(path, n, M, piece, window):
    """HOS_FULL_SQUARE on a streamed record: every piece carries a 2M-sample
    halo so the corner sums (offsets up to 2M) see the next pieces' samples;
    c3 over the whole square and B against the oracle."""
    hos = _hos()
    x = synth.quadratic_process(n, 700 + n).astype(np.float32)
    xh = torch.from_numpy(x)
    N = hos.default_nfft(M, window)
    print("case: square n=%d M=%d piece=%d window=%s path=%s" % (n, M, piece, window, path),
          flush=True)
    c3, B = hos.bispectrum_streamed(xh, M, piece=piece, nfft=N, window=window, path=path,
                                    full_square=True)
    torch.cuda.synchronize()
    c_ref, B_ref = oracle.bispectrum(x, M, N, window=window, full_square=True)
    e1, e2 = _err(c3.cpu().numpy(), c_ref), _err(B.cpu().numpy(), B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


@pytest.mark.parametrize("M,nfft,window,return_B", [
    (0, None, "parzen", True),      # lag 0 only
    (40, 81, "none", True),         # odd DFT size (3^4), no window
    (70, None, "parzen", False),    # c3 only
])
def test_edge_cases(M, nfft, window, return_B):
    hos = _hos()
    x = synth.iid_exp_centered(9000, 31 + M)
    print("case: n=9000 M=%d nfft=%s window=%s B=%s" % (M, nfft, window, return_B), flush=True)
    c3, B = hos.bispectrum_streamed(x, M, piece=4096, nfft=nfft, window=window,
                                    path="split_fp16", return_B=return_B)
    torch.cuda.synchronize()
    N = nfft or hos.default_nfft(M, window)
    c_ref, B_ref = oracle.bispectrum(x, M, N, window=window)
    assert _err(c3.cpu().numpy(), c_ref) < TOL["split_fp16"]
    if return_B:
        assert _err(B.cpu().numpy(), B_ref) < TOL["split_fp16"]
    else:
        assert B is None


def test_workload_sampled():
    """The streamed workload at its full size: n = 2^26 float32 quadratic
    process in pinned host memory, pieces of 2^22, M = 512, split FP16 (the
    configuration the benchmark times).  c3 at sampled lags against the
    oracle's sums; B against the in-memory call on the same record, which
    the streamed call equals up to the order of FP64 additions."""
    hos = _hos()
    x, cfg = synth.workload_streamed()
    M, N, piece = cfg["M"], cfg["nfft"], cfg["piece"]
    print("case: streamed workload n=%d M=%d piece=%d" % (x.size, M, piece), flush=True)
    xh = torch.from_numpy(x).pin_memory()
    cs, Bs = hos.bispectrum_streamed(xh, M, piece=piece, nfft=N, path="split_fp16")
    cm, Bm = hos.bispectrum(xh.cuda(), M, N, path="split_fp16")
    torch.cuda.synchronize()
    d = _err(Bs.cpu().numpy(), Bm.cpu().numpy())
    print("B streamed vs in-memory %.3e" % d)
    assert d < 1e-9
    rng = np.random.default_rng(5)
    w = rng.integers(-M, M + 1, (40, 2))
    w = w[np.abs(w[:, 0] - w[:, 1]) <= M]
    ref = oracle.c3_at(x, w[:, 0], w[:, 1])
    got = cs.cpu().numpy()[w[:, 0] + M, w[:, 1] + M]
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print("sampled rel err %.3e" % e)
    assert e < TOL["split_fp16"]
