"""GPU parity of the bispectrum path against the FP64 oracle.

Error measure: normwise relative error max|GPU - oracle| / max|oracle| over
the whole c3 hexagon (and over the N x N spectrum).  Bars: 1e-6 for the
FP32 path and 1e-5 for the split-precision paths.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-6, "split_fp16": 1e-5, "split_bf16": 1e-5}
PATHS = list(TOL)


def _hos():
    import paper_1805_11775_amd as hos
    assert hos.hos_device_check() == hos.HOS_OK, "no gfx950 device"
    return hos


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _run(x_np, M, nfft=None, window="parzen", path="fp32", center=True, dtype=None,
         full_square=False, pd_only=False):
    hos = _hos()
    t = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    print("case: n=%d M=%d nfft=%s window=%s path=%s dtype=%s square=%s pd=%s" %
          (t.numel(), M, nfft, window, path, t.dtype, full_square, pd_only), flush=True)
    c3, B = hos.bispectrum(t, M, nfft=nfft, window=window, path=path, center=center,
                           full_square=full_square, pd_only=pd_only)
    torch.cuda.synchronize()
    return c3.cpu().numpy(), B.cpu().numpy()


@pytest.mark.parametrize("path", PATHS)
def test_small_workload_exp_n2048_M64(path):
    """n = 2048 float64 centred Exp(1), M = 64, Parzen, 128-point DFT."""
    x, cfg = synth.workload_small_bispectrum()
    c3, B = _run(x, cfg["M"], cfg["nfft"], path=path)
    c3_ref, B_ref = oracle.bispectrum(x, cfg["M"], cfg["nfft"])
    e1, e2 = _rel(c3, c3_ref), _rel(B, B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,M", [(700, 0), (700, 1), (701, 5), (3001, 31), (3001, 32),
                                 (3001, 33), (4100, 95), (2500, 128), (3001, 160),
                                 (1537, 200), (700, 100), (1024, 96), (1025, 128),
                                 (2048, 129)])
def test_parity_grid(path, n, M):
    """Ragged lengths (not multiples of the 512-sample chunk, nor of the
    1024-sample chunk that 4-block split tiles stage), a record shorter than
    one such chunk, exact multiples, and lags below, at and above the
    32-block and 128-tile boundaries."""
    x = synth.quadratic_process(n, 1000 + n + M).astype(np.float32)
    c3, B = _run(x, M, path=path)
    c3_ref, B_ref = oracle.bispectrum(x, M, B.shape[0])
    e1, e2 = _rel(c3, c3_ref), _rel(B, B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path], (n, M, e1, e2)


@pytest.mark.parametrize("path", PATHS)
def test_gaussian_near_zero_cumulant(path):
    """i.i.d. Gaussian: c3 is pure sampling noise, the hardest case for a
    normwise bar; n = 65536, M = 64."""
    x = synth.iid_gauss(65536, 42).astype(np.float32)
    c3, _ = _run(x, 64, path=path)
    e = _rel(c3, oracle.c3_hexagon(x, 64))
    print("rel err c3 %.3e" % e)
    assert e < TOL[path]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,M", [(700, 1), (701, 5), (3001, 31), (3001, 32), (3001, 33),
                                 (4100, 95), (2500, 128), (3001, 160), (1537, 200),
                                 (700, 100), (1024, 96), (2048, 129)])
def test_full_square_grid(path, n, M):
    """HOS_FULL_SQUARE: c3 at every lag of the square, the corners
    |w1 - w2| > M included, element by element against the oracle's literal
    sums over the whole square; on the hexagon it is bitwise the default
    call's c3, and under the Parzen window (0 on the corners) B is too."""
    x = synth.quadratic_process(n, 2000 + n + M).astype(np.float32)
    c3, B = _run(x, M, path=path, full_square=True)
    c3_ref, B_ref = oracle.bispectrum(x, M, B.shape[0], full_square=True)
    e1, e2 = _rel(c3, c3_ref), _rel(B, B_ref)
    corner = oracle.span3(M) > M
    e3 = float(np.max(np.abs(c3 - c3_ref)[corner]) / np.max(np.abs(c3_ref))) if M > 0 else 0.0
    print("rel err c3 %.3e (corners %.3e) B %.3e" % (e1, e3, e2))
    assert e1 < TOL[path] and e2 < TOL[path], (n, M, e1, e2)
    assert M == 0 or np.max(np.abs(c3[corner])) > 0.0
    c3h, Bh = _run(x, M, path=path)
    assert np.array_equal(c3h[~corner], c3[~corner]) and np.all(c3h[corner] == 0.0)
    assert np.array_equal(Bh, B)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("window", ["none", "separable"])
def test_windows_nonzero_on_the_corners(path, window):
    """No window and the separable window weight the corners: B transforms
    the sample cumulant over the whole square (computed internally whatever
    the flags), against the oracle's; c3 stays on the hexagon unless asked."""
    n, M = 5003, 130
    x = synth.iid_exp_centered(n, 77).astype(np.float32)
    N = 270   # 2 * 3^3 * 5 >= 2M + 1
    c3, B = _run(x, M, nfft=N, window=window, path=path)
    c3_ref, B_ref = oracle.bispectrum(x, M, N, window=window)
    e1, e2 = _rel(c3, c3_ref), _rel(B, B_ref)
    print("rel err c3 %.3e B %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]
    assert np.all(c3[oracle.span3(M) > M] == 0.0)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [128, 135, 150, 250])
def test_principal_domain_only(path, N):
    """HOS_PD_ONLY: B packed on 0 <= k2 <= k1, k1 + k2 < N/2 in row-major
    order, bitwise the full grid's values there, and against the oracle."""
    x = synth.quadratic_process(9000, 31).astype(np.float32)
    M = 60
    _, Bfull = _run(x, M, nfft=N, path=path)
    _, Bpd = _run(x, M, nfft=N, path=path, pd_only=True)
    k1, k2 = oracle.pd_indices(N)
    assert Bpd.shape == (len(k1),)
    assert np.array_equal(Bpd, Bfull[k1, k2])
    B_ref = oracle.bispectrum_pd(x, M, N)
    assert _rel(Bpd, B_ref) < TOL[path]


@pytest.mark.timeout(600)
def test_headline_full_square_against_oracle():
    """n = 2^20 float32 quadratic process, M = 512, 1024-point DFT on the
    split-FP16 path: c3 over the whole square ((2M+1)^2 lags: the hexagon
    the benchmark times plus the corners) and B at every frequency, element
    by element against the oracle (about 1.1e12 FP64 products)."""
    x, cfg = synth.workload_long_bispectrum()
    M, N = cfg["M"], cfg["nfft"]
    c3, B = _run(x, M, N, path="split_fp16", full_square=True)
    print("oracle: full square at n=%d M=%d" % (x.size, M), flush=True)
    c3_ref, B_ref = oracle.bispectrum(x, M, N, full_square=True)
    hexagon = oracle.span3(M) <= M
    e_hex = float(np.max(np.abs(c3 - c3_ref)[hexagon]) / np.max(np.abs(c3_ref[hexagon])))
    e_sq, e_B = _rel(c3, c3_ref), _rel(B, B_ref)
    print("rel err c3 hexagon %.3e square %.3e B %.3e" % (e_hex, e_sq, e_B), flush=True)
    assert e_hex < 1e-5 and e_sq < 1e-5 and e_B < 1e-5
    # the benchmark's call (hexagon) returns bitwise the same hexagon
    c3h, Bh = _run(x, M, N, path="split_fp16")
    assert np.array_equal(c3h[hexagon], c3[hexagon]) and np.array_equal(Bh, B)


@pytest.mark.parametrize("window", ["none", "parzen", "separable"])
def test_window_and_nfft_variants(window):
    x = synth.iid_exp_centered(1500, 7)
    M = 20
    for nfft in ([45, 48, 64] if window == "none" else [40, 48, 60]):
        c3, B = _run(x, M, nfft=nfft, window=window)
        _, B_ref = oracle.bispectrum(x, M, nfft, window=window)
        assert _rel(B, B_ref) < 1e-6, nfft


def test_impulse_uncentered_closed_form():
    """x = A delta_{t0}, no mean removal: c3 = A^3/n at the origin only and
    the spectrum is flat."""
    n, M, A = 4000, 40, 3.0
    x = np.zeros(n)
    x[1234] = A
    c3, B = _run(x, M, nfft=80, center=False)
    expect = np.zeros_like(c3)
    expect[M, M] = A ** 3 / n
    assert np.max(np.abs(c3 - expect)) < 1e-6 * A ** 3 / n
    assert np.max(np.abs(B - A ** 3 / n)) < 1e-6 * A ** 3 / n


def test_constant_series_is_zero():
    c3, B = _run(np.full(3000, 2.5), 50)
    assert np.max(np.abs(c3)) == 0.0 and np.max(np.abs(B)) == 0.0


def test_deterministic_and_workspace_independent():
    """Bitwise-equal reruns; a NaN-poisoned workspace changes nothing."""
    hos = _hos()
    x = torch.from_numpy(synth.quadratic_process(200000, 3).astype(np.float32)).cuda()
    M, nfft = 256, 512
    c3a, Ba = hos.bispectrum(x, M, nfft=nfft, path="split_fp16")
    nb = hos.hos_bispectrum_workspace(x.numel(), M, nfft, hos.HOS_PATH_SPLIT_FP16)
    ws = torch.full((nb,), 0xFF, dtype=torch.uint8, device="cuda")  # NaN bytes
    c3b, Bb = hos.bispectrum(x, M, nfft=nfft, path="split_fp16", workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(c3a, c3b) and torch.equal(Ba, Bb)
    assert not torch.isnan(c3a).any()


@pytest.mark.parametrize("path", PATHS)
def test_long_workload_sampled(path):
    """n = 2^20 float32 quadratic process, M = 512, 1024-point DFT (the
    benchmark shape and launch configuration): sampled lags against the
    oracle, spectrum symmetries at every frequency, and sampled frequencies
    against a direct DFT of the returned c3."""
    x, cfg = synth.workload_long_bispectrum()
    M, N = cfg["M"], cfg["nfft"]
    c3, B = _run(x, M, N, path=path)
    rng = np.random.default_rng(5)
    w1 = rng.integers(-M, M + 1, 200)
    w2 = np.clip(w1 + rng.integers(-M, M + 1, 200), -M, M)
    orbit = np.array([[1, 2], [2, 1], [-1, 1], [1, -1], [-2, -1], [-1, -2], [0, 0],
                      [M, 0], [0, M], [M, M], [-M, -M], [M, 1], [32, 32], [64, 0]])
    w1 = np.concatenate([w1, orbit[:, 0]])
    w2 = np.concatenate([w2, orbit[:, 1]])
    ref = oracle.c3_at(x, w1, w2)
    ref[np.abs(w1 - w2) > M] = 0.0
    got = c3[w1 + M, w2 + M]
    scale = np.max(np.abs(c3))
    e = np.max(np.abs(got - ref)) / scale
    print("sampled rel err c3 %.3e" % e)
    assert e < TOL[path]
    assert abs(scale - np.max(np.abs(ref))) / scale < 1e-3  # the max is in the sample
    # c3 symmetries hold exactly (one table entry per orbit)
    assert np.array_equal(c3, c3.T)
    # spectrum symmetries at every frequency
    k = np.arange(N)
    tol = 1e-9 * np.max(np.abs(B))
    assert np.max(np.abs(B - B.T)) < tol
    assert np.max(np.abs(B - np.conj(B[(-k[:, None]) % N, (-k[None, :]) % N]))) < tol
    # the DFT stage: sampled frequencies against a direct sum over the lags
    W = oracle.window3(M)
    lag = np.arange(-M, M + 1)
    cw = W * c3
    for k1, k2 in [(0, 0), (1, 2), (17, 300), (511, 512), (1023, 5)]:
        e = np.exp(-2j * np.pi * (k1 * lag[:, None] + k2 * lag[None, :]) / N)
        assert abs(np.sum(cw * e) - B[k1, k2]) < 1e-10 * np.max(np.abs(B))


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_max_lag_c3_only(path):
    """M = 8192, the largest lag of the entry point (c3 only: a spectrum
    needs N >= 2M and N <= 4096).  n = 20000, so most lags reach past the
    record; c3 at sampled lags against the oracle's sums."""
    hos = _hos()
    M, n = 8192, 20000
    x = synth.quadratic_process(n, 91).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    print("case: max lag n=%d M=%d path=%s c3 only" % (n, M, path), flush=True)
    c3, B = hos.bispectrum(t, M, path=path, return_B=False)
    torch.cuda.synchronize()
    assert B is None
    rng = np.random.default_rng(12)
    w = rng.integers(-M, M + 1, (300, 2))
    w = w[np.abs(w[:, 0] - w[:, 1]) <= M]
    w = np.concatenate([w, [[0, 0], [1, 2], [2, 1], [-1, 1], [M, M], [-M, 0], [5000, 4999]]])
    ref = oracle.c3_at(x, w[:, 0], w[:, 1])
    got = c3[torch.from_numpy(w[:, 0] + M).cuda(), torch.from_numpy(w[:, 1] + M).cuda()]
    e = _rel(got.cpu().numpy(), ref)
    print("sampled rel err c3 %.3e" % e)
    assert e < TOL[path]


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_max_dft(path):
    """N = 4096, the largest DFT, at M = 2048 (n = 8000): c3 at sampled lags
    against the oracle, and the spectrum's symmetries B(k1, k2) = B(k2, k1)
    = conj B(-k1, -k2) (mod N) at sampled points, which hold for the
    windowed c3 at any size."""
    hos = _hos()
    M, n, N = 2048, 8000, 4096
    x = synth.iid_exp_centered(n, 92).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    print("case: max dft n=%d M=%d N=%d path=%s" % (n, M, N, path), flush=True)
    c3, B = hos.bispectrum(t, M, nfft=N, path=path)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    w = rng.integers(-M, M + 1, (300, 2))
    w = w[np.abs(w[:, 0] - w[:, 1]) <= M]
    w = np.concatenate([w, [[0, 0], [M, M], [-M, 0]]])
    ref = oracle.c3_at(x, w[:, 0], w[:, 1])
    got = c3[torch.from_numpy(w[:, 0] + M).cuda(), torch.from_numpy(w[:, 1] + M).cuda()]
    e = _rel(got.cpu().numpy(), ref)
    print("sampled rel err c3 %.3e" % e)
    assert e < TOL[path]
    k = torch.from_numpy(rng.integers(0, N, (4000, 2))).cuda()
    b = B[k[:, 0], k[:, 1]]
    bt = B[k[:, 1], k[:, 0]]
    bc = B[(-k[:, 0]) % N, (-k[:, 1]) % N].conj()
    scale = float(B.abs().max())
    s1 = float((b - bt).abs().max()) / scale
    s2 = float((b - bc).abs().max()) / scale
    print("symmetry %.3e %.3e" % (s1, s2))
    assert s1 < 1e-12 and s2 < 1e-12


@pytest.mark.parametrize("path,peak", [("split_fp16", 2.5166e15), ("fp32", 157.3e12)])
def test_mfma_rate_probe(path, peak):
    """The measurement helper behind the benchmark's matrix-core ceiling: a
    positive rate below the published dense peak."""
    hos = _hos()
    r = hos.mfma_rate(path, 1 << 16)
    print("mfma rate %s: %.1f TFLOP/s in %.2f ms" % (path, r["tflops"], r["ms"]))
    assert r["ms"] > 0.0 and 0.05 * peak < r["tflops"] * 1e12 < 1.02 * peak
