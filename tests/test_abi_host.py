"""Host-side checks of the C ABI: symbols, validation before any HIP call,
and the contraction's work split (replayed on the CPU by the library)."""
import ctypes
import os
import re

import pytest

import oracle
import paper_1805_11775_amd as hos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hos_\w+)\s*\(", txt, flags=re.M)
    return names


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert "hos_bispectrum" in names and len(names) >= 7
    lib = ctypes.CDLL(hos.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strerror():
    assert hos.hos_version() == 10000
    for code in (0, -1, -2, -3, -4, -5, -6, 7):
        assert isinstance(hos.hos_strerror(code), str)


FAKE = 0x10000  # any aligned non-null address; validation fails before use


@pytest.mark.parametrize("kw,code", [
    (dict(n=1), hos.HOS_EINVAL),
    (dict(M=-1), hos.HOS_EINVAL),
    (dict(M=100, n=100), hos.HOS_EINVAL),
    (dict(path=3), hos.HOS_EINVAL),
    (dict(window=3), hos.HOS_EINVAL),
    (dict(dtype=5), hos.HOS_EINVAL),
    (dict(flags=8), hos.HOS_EINVAL),
    (dict(nfft=127), hos.HOS_EINVAL),        # < 2M with Parzen
    (dict(nfft=7 * 37), hos.HOS_EINVAL),     # not 2^a 3^b 5^c
    (dict(nfft=128, window=0), hos.HOS_EINVAL),  # < 2M+1 without window
    (dict(x=None), hos.HOS_EINVAL),
    (dict(x=FAKE + 2), hos.HOS_EINVAL),      # misaligned float32
    (dict(ws=FAKE + 64), hos.HOS_EINVAL),    # workspace not 256-aligned
    (dict(c3=None, B=None), hos.HOS_EINVAL),
    (dict(ws_bytes=16), hos.HOS_EWORKSPACE),
    (dict(n=(1 << 31) + 1, M=64), hos.HOS_EINVAL),      # beyond the series limit
    (dict(flags=hos.HOS_FULL_SQUARE, ws_bytes=16), hos.HOS_EWORKSPACE),   # flag accepted
    (dict(flags=hos.HOS_PD_ONLY | hos.HOS_FULL_SQUARE | hos.HOS_NO_CENTER, ws_bytes=16),
     hos.HOS_EWORKSPACE),
    (dict(flags=16), hos.HOS_EINVAL),                   # a batch-plan flag
])
def test_validation_before_device(kw, code):
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=4096, M=64, window=hos.HOS_WIN_PARZEN,
             nfft=128, path=hos.HOS_PATH_FP32, flags=0, c3=FAKE, B=FAKE, ws=FAKE,
             ws_bytes=1 << 40, stream=None)
    a.update(kw)
    st = hos.hos_bispectrum(a["x"], a["dtype"], a["n"], a["M"], a["window"], a["nfft"],
                            a["path"], a["flags"], a["c3"], a["B"], a["ws"],
                            a["ws_bytes"], a["stream"])
    assert st == code


@pytest.mark.parametrize("kw,code", [
    (dict(n=1), hos.HOS_EINVAL),
    (dict(M=100, n=100), hos.HOS_EINVAL),
    (dict(path=3), hos.HOS_EINVAL),
    (dict(window=3), hos.HOS_EINVAL),
    (dict(dtype=5), hos.HOS_EINVAL),
    (dict(flags=8), hos.HOS_EINVAL),
    (dict(nfft=127), hos.HOS_EINVAL),
    (dict(x=None), hos.HOS_EINVAL),
    (dict(x=FAKE + 2), hos.HOS_EINVAL),
    (dict(B=FAKE + 8), hos.HOS_EINVAL),
    (dict(c3=None, B=None), hos.HOS_EINVAL),
    # beyond the fixed scratch: 2^22 samples at M = 512 need ~470 MiB
    (dict(n=1 << 22, M=512, nfft=1024, path=hos.HOS_PATH_SPLIT_FP16), hos.HOS_ESCRATCH),
    (dict(n=1 << 21, M=512, nfft=1024, path=hos.HOS_PATH_SPLIT_FP16), hos.HOS_ESCRATCH),
])
def test_noalloc_validation_before_device(kw, code):
    """The non-allocating entry point rejects bad arguments, and requests
    beyond its fixed scratch, on the host before any HIP call."""
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=4096, M=64, window=hos.HOS_WIN_PARZEN,
             nfft=128, path=hos.HOS_PATH_FP32, flags=0, c3=FAKE, B=FAKE, stream=None)
    a.update(kw)
    st = hos.hos_bispectrum_noalloc(a["x"], a["dtype"], a["n"], a["M"], a["window"],
                                    a["nfft"], a["path"], a["flags"], a["c3"], a["B"],
                                    a["stream"])
    assert st == code
    assert "scratch" in hos.hos_strerror(hos.HOS_ESCRATCH)


def test_noalloc_scratch_covers_the_headline_shape():
    # the largest single-series shape the benchmark runs fits the fixed scratch
    for path in (hos.HOS_PATH_FP32, hos.HOS_PATH_SPLIT_FP16, hos.HOS_PATH_SPLIT_BF16):
        assert hos.hos_bispectrum_workspace(1 << 20, 512, 1024, path) <= \
            hos.HOS_NOALLOC_SCRATCH_BYTES


@pytest.mark.parametrize("n,M,N,path", [(1 << 20, 512, 1024, 1), (5000, 33, 72, 0),
                                         (4096, 100, 200, 2)])
def test_workspace_flags(n, M, N, path):
    """The corner rows are in every layout (their need depends on the window,
    which the query does not take); the principal-domain output stages the
    full grid in the workspace."""
    base = hos.hos_bispectrum_workspace(n, M, N, path)
    assert hos.hos_bispectrum_workspace(n, M, N, path, hos.HOS_FULL_SQUARE) == base
    pd = hos.hos_bispectrum_workspace(n, M, N, path, hos.HOS_PD_ONLY)
    assert base + 16 * N * N <= pd <= base + 16 * N * N + 256
    assert hos.hos_bispectrum_workspace(n, M, 0, path, hos.HOS_PD_ONLY) == \
        hos.hos_bispectrum_workspace(n, M, 0, path)


@pytest.mark.parametrize("path,iters", [(7, 100), (hos.HOS_PATH_SPLIT_FP16, 0),
                                        (hos.HOS_PATH_FP32, (1 << 24) + 1)])
def test_mfma_rate_validation_before_device(path, iters):
    ms, fl = ctypes.c_float(0.0), ctypes.c_double(0.0)
    assert hos.lib().hos_mfma_rate(path, iters, ctypes.byref(ms), ctypes.byref(fl),
                                   None) == hos.HOS_EINVAL
    assert hos.lib().hos_mfma_rate(hos.HOS_PATH_SPLIT_FP16, 100, None, ctypes.byref(fl),
                                   None) == hos.HOS_EINVAL


def test_pd_count_matches_the_oracle():
    for N in (2, 3, 4, 7, 16, 33, 128, 1024):
        assert hos.pd_count(N) == len(oracle.pd_indices(N)[0])


def test_workspace_query():
    b = hos.hos_bispectrum_workspace(1 << 20, 512, 1024, hos.HOS_PATH_SPLIT_FP16)
    b32 = hos.hos_bispectrum_workspace(1 << 20, 512, 1024, hos.HOS_PATH_FP32)
    assert b > b32 > (1 << 20) * 20
    with pytest.raises(hos.HosError):
        hos.hos_bispectrum_workspace(10, 10, 0, 0)


@pytest.mark.parametrize("n,M,path", [
    (2048, 64, 0), (1 << 20, 512, 1), (1 << 20, 512, 0), (5000, 33, 2),
    (65536, 256, 1), (1025, 128, 0), (70001, 300, 1), (3000, 1, 0), (600, 95, 2),
    (1 << 16, 1000, 0),
])
def test_schedule_covers_every_chunk_once(n, M, path):
    info = hos.hos_c3_plan_info(n, M, path)
    owner, slot, rslot = hos.hos_c3_schedule(n, M, path)
    assert len(owner) == info["TR"] * (info["TR"] + 1) // 2 * info["C"]
    assert min(owner) >= 0, "a chunk is unowned (-1) or owned twice (-2)"
    assert max(owner) < info["G"]
    assert min(slot) >= 0 and max(slot) < info["G"] * info["smax"]
    assert slot == rslot, "reduce reads a different slot than the kernel writes"
    # every workgroup processes at least one chunk
    assert len(set(owner)) == info["G"]


@pytest.mark.parametrize("kw,code", [
    (dict(n=1), hos.HOS_EINVAL),
    (dict(M=128, nfft=256), hos.HOS_EINVAL),   # beyond the fourth-order lag limit
    (dict(M=-1), hos.HOS_EINVAL),
    (dict(M=40, n=40), hos.HOS_EINVAL),
    (dict(path=3), hos.HOS_EINVAL),
    (dict(window=3), hos.HOS_EINVAL),
    (dict(flags=2), hos.HOS_EINVAL),
    (dict(nfft=95), hos.HOS_EINVAL),          # < 2M with Parzen
    (dict(nfft=96, window=0), hos.HOS_EINVAL),  # < 2M+1 without window
    (dict(nfft=7 * 16), hos.HOS_EINVAL),      # not 2^a 3^b 5^c
    (dict(nfft=600), hos.HOS_EINVAL),         # N^3 grid beyond 512 per axis
    (dict(x=FAKE + 4, dtype=hos.HOS_F64), hos.HOS_EINVAL),
    (dict(T=FAKE + 8), hos.HOS_EINVAL),       # complex128 needs 16-byte alignment
    (dict(c4=None, T=None), hos.HOS_EINVAL),
    (dict(ws_bytes=1024), hos.HOS_EWORKSPACE),
    # windows nonzero where the span exceeds M: outside the contraction's region
    (dict(window=hos.HOS_WIN_NONE, nfft=100), hos.HOS_EUNSUPPORTED),
    (dict(window=hos.HOS_WIN_PARZEN_SEPARABLE), hos.HOS_EUNSUPPORTED),
    (dict(flags=hos.HOS_FULL_SQUARE), hos.HOS_EINVAL),
])
def test_trispectrum_validation_before_device(kw, code):
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=1 << 18, M=48, window=hos.HOS_WIN_PARZEN,
             nfft=96, path=hos.HOS_PATH_SPLIT_FP16, flags=0, c4=FAKE, T=FAKE, ws=FAKE,
             ws_bytes=1 << 40, stream=None)
    a.update(kw)
    st = hos.hos_trispectrum(a["x"], a["dtype"], a["n"], a["M"], a["window"], a["nfft"],
                             a["path"], a["flags"], a["c4"], a["T"], a["ws"],
                             a["ws_bytes"], a["stream"])
    assert st == code


@pytest.mark.parametrize("n,M,path", [
    (1 << 18, 48, 1), (1 << 18, 48, 0), (700, 0, 0), (701, 31, 2), (3001, 32, 1),
    (5000, 127, 0), (1 << 22, 127, 1), (513, 5, 2), (100000, 63, 1),
])
def test_c4_plan(n, M, path):
    """Pair count and blocking, window reach, and the sample-axis split:
    S ranges of CPS chunks, every range non-empty, together covering C."""
    info = hos.hos_c4_plan_info(n, M, path)
    assert info["P"] == (M + 1) * (M + 2) // 2
    assert info["RB"] == -(-info["P"] // 32)
    assert info["NCB"] == -(-(M + 1) // 32)
    assert info["WX"] >= 32 * info["NCB"] + 16 and info["WX"] % 64 == 0
    assert info["C"] == -(-n // 512)
    S, cps, C = info["S"], info["CPS"], info["C"]
    assert (S - 1) * cps < C <= S * cps
    assert info["ws_bytes"] == hos.hos_trispectrum_workspace(n, M, 0, path)
    assert hos.hos_trispectrum_workspace(n, M, hos.default_nfft(M), path) > info["ws_bytes"]


@pytest.mark.parametrize("kw,code", [
    (dict(M=41), hos.HOS_EINVAL),              # beyond the order-five lag limit
    (dict(nfft=120, M=40), hos.HOS_EINVAL),    # beyond the 4-D DFT limit
    (dict(nfft=20, M=12), hos.HOS_EINVAL),     # < 2M with Parzen
    (dict(window=3), hos.HOS_EINVAL),
    (dict(c5=None, Q=None), hos.HOS_EINVAL),
    (dict(Q=FAKE + 8), hos.HOS_EINVAL),
    (dict(ws_bytes=16), hos.HOS_EWORKSPACE),
    (dict(window=hos.HOS_WIN_NONE, nfft=18), hos.HOS_EUNSUPPORTED),
    (dict(window=hos.HOS_WIN_PARZEN_SEPARABLE), hos.HOS_EUNSUPPORTED),
])
def test_cumulant5_validation_before_device(kw, code):
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=4096, M=8, window=hos.HOS_WIN_PARZEN,
             nfft=16, path=hos.HOS_PATH_SPLIT_FP16, flags=0, c5=FAKE, Q=FAKE, ws=FAKE,
             ws_bytes=1 << 40)
    a.update(kw)
    st = hos.lib().hos_cumulant5(a["x"], a["dtype"], a["n"], a["M"], a["window"], a["nfft"],
                                 a["path"], a["flags"], a["c5"], a["Q"], a["ws"],
                                 a["ws_bytes"], None)
    assert st == code


def test_c5_plan():
    info = hos.hos_c5_plan_info(1 << 18, 24, hos.HOS_PATH_SPLIT_FP16)
    assert info["P"] == 25 * 26 * 27 // 6 and info["RB"] == (info["P"] + 31) // 32
    assert info["NCB"] == 1 and info["WX"] >= 32 * info["NCB"] + 16
    assert info["S"] * info["CPS"] >= info["C"]


@pytest.mark.parametrize("kw,code", [
    (dict(piece=4096 + 512), hos.HOS_EINVAL),   # not a multiple of 1024
    (dict(piece=2048), hos.HOS_EINVAL),         # below 4096
    (dict(piece=4096, M=5000, nfft=10000), hos.HOS_EINVAL),   # shorter than M
    (dict(x=None), hos.HOS_EINVAL),
    (dict(c3=None, B=None), hos.HOS_EINVAL),
    (dict(ws_bytes=1000), hos.HOS_EWORKSPACE),
    (dict(B=None, nfft=-1), hos.HOS_EINVAL),
    (dict(nfft=100), hos.HOS_EINVAL),          # below 2M with a window
    (dict(flags=hos.HOS_FULL_SQUARE, ws_bytes=1000), hos.HOS_EWORKSPACE),   # accepted
    (dict(flags=hos.HOS_PD_ONLY), hos.HOS_EINVAL),   # one series' call only
])
def test_streamed_validation_before_device(kw, code):
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=1 << 20, M=64, window=hos.HOS_WIN_PARZEN, nfft=128,
             path=hos.HOS_PATH_FP32, flags=0, piece=1 << 16, c3=FAKE, B=FAKE, ws=FAKE,
             ws_bytes=1 << 40)
    a.update(kw)
    st = hos.lib().hos_bispectrum_streamed(a["x"], a["dtype"], a["n"], a["M"], a["window"],
                                          a["nfft"], a["path"], a["flags"], a["piece"], a["c3"],
                                          a["B"], a["ws"], a["ws_bytes"], None)
    assert st == code


def test_streamed_workspace_independent_of_n():
    import ctypes
    sizes = []
    for n in (1 << 22, 1 << 26, 1 << 30):
        b = ctypes.c_size_t(0)
        assert hos.lib().hos_bispectrum_streamed_workspace(n, 512, 1024, 1, 0, 1 << 20,
                                                          ctypes.byref(b)) == 0
        sizes.append(b.value)
    assert sizes[0] == sizes[1] == sizes[2]
