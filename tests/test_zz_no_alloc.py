"""GPU check of hos_bispectrum_noalloc, the entry point that allocates
nothing (its workspace is the library's fixed per-device scratch array).

Two calls in a row through the C ABI, the second on a smaller input, each
compared with hos_bispectrum on a caller workspace: both run the same
kernels on the same plan with fixed-order reductions, so the results must be
bitwise equal.  The first case is also held to the FP64 oracle (split-FP16
bar, 1e-5 normwise).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hos():
    import paper_1805_11775_amd as hos
    assert hos.hos_device_check() == hos.HOS_OK, "no gfx950 device"
    return hos


def _pair(hos, x_np, M, nfft, path, window, want_c3=True, want_B=True):
    """(c3, B) from hos_bispectrum_noalloc and from hos_bispectrum."""
    dev = torch.device("cuda")
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev)
    dt = hos.HOS_F64 if x.dtype == torch.float64 else hos.HOS_F32
    n = x.numel()
    pth = hos.PATHS[path]
    win = hos.WINDOWS[window]
    stream = hos._stream_handle(dev)
    out = []
    for noalloc in (True, False):
        c3 = torch.full((2 * M + 1, 2 * M + 1), float("nan"), dtype=torch.float64,
                        device=dev) if want_c3 else None
        B = torch.full((nfft, nfft), complex("nan"), dtype=torch.complex128,
                       device=dev) if want_B else None
        c3p = c3.data_ptr() if c3 is not None else None
        Bp = B.data_ptr() if B is not None else None
        print("case: noalloc=%s n=%d M=%d nfft=%d path=%s window=%s c3=%s B=%s" %
              (noalloc, n, M, nfft, path, window, want_c3, want_B), flush=True)
        if noalloc:
            st = hos.hos_bispectrum_noalloc(x.data_ptr(), dt, n, M, win,
                                            nfft if want_B else 0, pth, 0, c3p, Bp, stream)
        else:
            wsb = hos.hos_bispectrum_workspace(n, M, nfft if want_B else 0, pth)
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            st = hos.hos_bispectrum(x.data_ptr(), dt, n, M, win, nfft if want_B else 0, pth,
                                    0, c3p, Bp, ws.data_ptr(), wsb, stream)
        assert st == hos.HOS_OK, hos.hos_strerror(st)
        torch.cuda.synchronize()
        out.append((c3.cpu().numpy() if c3 is not None else None,
                    B.cpu().numpy() if B is not None else None))
    return out[0], out[1]


def _same(a, b):
    assert (a is None) == (b is None)
    if a is not None:
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), \
            "non-allocating call differs from hos_bispectrum"


def test_noalloc_two_calls_second_smaller():
    hos = _hos()
    # first call: 3 x 2^16 samples, M = 200 (several 4-block tiles, ragged)
    x1 = synth.quadratic_process(3 * 65536 + 77, 180511790).astype(np.float32)
    (c3a, Ba), (c3b, Bb) = _pair(hos, x1, 200, 400, "split_fp16", "parzen")
    _same(c3a, c3b)
    _same(Ba, Bb)
    c3r, Br = oracle.bispectrum(x1.astype(np.float64), 200, 400)
    e1 = np.max(np.abs(c3a - c3r)) / np.max(np.abs(c3r))
    e2 = np.max(np.abs(Ba - Br)) / np.max(np.abs(Br))
    print("oracle rel err c3 %.3e B %.3e" % (e1, e2), flush=True)
    assert e1 < 1e-5 and e2 < 1e-5
    # second call, smaller: the scratch keeps the first call's contents
    x2 = synth.iid_exp_centered(5001, 180511791)
    (c3a, Ba), (c3b, Bb) = _pair(hos, x2, 33, 72, "fp32", "parzen")
    _same(c3a, c3b)
    _same(Ba, Bb)
    c3r, Br = oracle.bispectrum(x2, 33, 72)
    assert np.max(np.abs(c3a - c3r)) / np.max(np.abs(c3r)) < 1e-6


@pytest.mark.parametrize("path", ["fp32", "split_bf16"])
def test_noalloc_single_outputs_and_headline_shape(path):
    hos = _hos()
    # B only, then c3 only, at the benchmark's headline shape (fits the scratch)
    x, cfg = synth.workload_long_bispectrum()
    (c3a, Ba), (c3b, Bb) = _pair(hos, x, cfg["M"], cfg["nfft"], path, "parzen",
                                 want_c3=False)
    _same(Ba, Bb)
    x2 = synth.iid_gauss(4097, 180511792)
    (c3a, Ba), (c3b, Bb) = _pair(hos, x2, 64, 128, path, "none", want_B=False)
    _same(c3a, c3b)


def test_noalloc_rejects_oversize_without_touching_the_device():
    hos = _hos()
    x = torch.zeros(1 << 22, dtype=torch.float32, device="cuda")
    c3 = torch.zeros((1025, 1025), dtype=torch.float64, device="cuda")
    st = hos.hos_bispectrum_noalloc(x.data_ptr(), hos.HOS_F32, x.numel(), 512,
                                    hos.HOS_WIN_PARZEN, 0, hos.HOS_PATH_SPLIT_FP16, 0,
                                    c3.data_ptr(), None, hos._stream_handle(x.device))
    assert st == hos.HOS_ESCRATCH
    torch.cuda.synchronize()
    assert float(c3.abs().max()) == 0.0
