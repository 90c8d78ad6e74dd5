"""HIP-graph capture of the single-series entry points.

hos_bispectrum and hos_trispectrum only enqueue kernels on the caller's
stream: no allocation, no host synchronisation and no memset node.  So a call
can be captured into a graph and replayed (a serving loop's launch overhead
then goes).  Every replay must equal an eager call on the same input bit for
bit, since the reductions run in a fixed order.  The tests check this over
several replays, with the input changed between them and with other eager
work and synchronisations in between.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hos():
    import paper_1805_11775_amd as hos
    assert hos.hos_device_check() == hos.HOS_OK, "no gfx950 device"
    return hos


def _capture(call):
    """Warm up on a side stream (default priority), then capture one call."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    return g


def _replays_match_eager(hos, x, inputs, outs, call):
    """Replay the captured call once per input (copied into x) and compare
    every output with an eager call on the same input."""
    g = _capture(lambda: call(outs))
    eager = [torch.empty_like(o) for o in outs]
    for k, xin in enumerate(inputs):
        print("replay %d" % k, flush=True)
        x.copy_(xin)
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outs]
        # eager work between replays: the same call into other buffers, and
        # an unrelated torch op on the stream
        call(eager)
        torch.cuda.synchronize()
        _ = (x * 2.0).sum().item()
        for a, b in zip(got, eager):
            assert torch.equal(a, b), "replay %d differs from the eager call" % k


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_bispectrum_graph_replays_match_eager(path):
    hos = _hos()
    n, M, N = 1 << 16, 64, 128
    pth = hos.PATHS[path]
    print("case: bispectrum n=%d M=%d N=%d path=%s" % (n, M, N, path), flush=True)
    inputs = [torch.from_numpy(synth.quadratic_process(n, s).astype(np.float32)).cuda()
              for s in (11, 12, 13)]
    x = inputs[0].clone()
    wsb = hos.hos_bispectrum_workspace(n, M, N, pth)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    outs = [torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64, device="cuda"),
            torch.empty((N, N), dtype=torch.complex128, device="cuda")]

    def call(o):
        st = hos.hos_bispectrum(x.data_ptr(), hos.HOS_F32, n, M, hos.HOS_WIN_PARZEN, N, pth, 0,
                                o[0].data_ptr(), o[1].data_ptr(), ws.data_ptr(), wsb,
                                hos._stream_handle(x.device))
        assert st == hos.HOS_OK

    _replays_match_eager(hos, x, inputs, outs, call)


def test_trispectrum_graph_replays_match_eager():
    hos = _hos()
    n, M, N = 1 << 15, 16, 32
    pth = hos.PATHS["split_fp16"]
    print("case: trispectrum n=%d M=%d N=%d" % (n, M, N), flush=True)
    inputs = [torch.from_numpy(synth.cubic_process(n, s).astype(np.float32)).cuda()
              for s in (21, 22, 23)]
    x = inputs[0].clone()
    wsb = hos.hos_trispectrum_workspace(n, M, N, pth)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    outs = [torch.empty((2 * M + 1,) * 3, dtype=torch.float64, device="cuda"),
            torch.empty((N, N, N), dtype=torch.complex128, device="cuda")]

    def call(o):
        st = hos.hos_trispectrum(x.data_ptr(), hos.HOS_F32, n, M, hos.HOS_WIN_PARZEN, N, pth,
                                 0, o[0].data_ptr(), o[1].data_ptr(), ws.data_ptr(), wsb,
                                 hos._stream_handle(x.device))
        assert st == hos.HOS_OK

    _replays_match_eager(hos, x, inputs, outs, call)
