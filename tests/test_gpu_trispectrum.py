"""GPU parity of the trispectrum path against the FP64 oracle.

Error measure for c4: max|GPU - oracle| over the whole cube, divided by the
fourth sample moment at the origin, m4(0,0,0) = (1/n) sum x~^4.  That moment
bounds |m4| at every lag (Hoelder), so the contraction's rounding -- the
only reduced-precision step -- is at most a path-dependent multiple of it;
the c2 corrections are FP64 on every path.  Bars: 1e-6 for the FP32 path and
1e-5 for the split paths, as for the bispectrum.  Spectra are compared
normwise against max|T_oracle|.
"""
import functools

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


def _run(x_np, M, nfft=None, window="parzen", path="fp32", center=True, return_T=True):
    hos = _hos()
    t = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda")
    print("case: n=%d M=%d nfft=%s window=%s path=%s dtype=%s" %
          (t.numel(), M, nfft, window, path, t.dtype), flush=True)
    c4, T = hos.trispectrum(t, M, nfft=nfft, window=window, path=path, center=center,
                            return_T=return_T)
    torch.cuda.synchronize()
    return c4.cpu().numpy(), (T.cpu().numpy() if T is not None else None)


def _m4_origin(x, center=True):
    return float(oracle.m4_at(x, [0], [0], [0], centered=center)[0])


def _err(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / scale)


@functools.lru_cache(maxsize=None)
def _oracle_case(n, M, seed, want_T):
    x = synth.cubic_process(n, seed).astype(np.float32)
    if want_T:
        N = _hos().default_nfft(M)
        c, T = oracle.trispectrum(x, M, N)
    else:
        c, T = oracle.c4_support(x, M), None
    return x, c, T


@pytest.mark.parametrize("path", PATHS)
def test_workload_shape_small_exp(path):
    """Centred Exp(1), n = 3000, M = 20, Parzen, 48^3 DFT: every lag and
    every frequency."""
    x = synth.iid_exp_centered(3000, 21)
    c4, T = _run(x, 20, 48, path=path)
    c_ref, T_ref = oracle.trispectrum(x, 20, 48)
    e1 = _err(c4, c_ref, _m4_origin(x))
    e2 = _err(T, T_ref, np.max(np.abs(T_ref)))
    print("rel err c4 %.3e T %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,M", [(700, 0), (700, 1), (701, 5), (1500, 31), (1500, 32),
                                 (2100, 33), (1300, 63), (1200, 64), (900, 100)])
def test_parity_grid(path, n, M):
    """Ragged lengths and lags below, at and above the 32-pair / 32-column
    block boundaries and the staged-window sizes."""
    x, c_ref, T_ref = _oracle_case(n, M, 2000 + n + M, True)
    c4, T = _run(x, M, T_ref.shape[0], path=path)
    e1 = _err(c4, c_ref, _m4_origin(x))
    e2 = _err(T, T_ref, np.max(np.abs(T_ref)))
    print("rel err c4 %.3e T %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path], (n, M, e1, e2)


@pytest.mark.parametrize("path", PATHS)
def test_max_lag(path):
    """M = 127, the largest lag of the fourth-order path (4 column blocks)."""
    x, c_ref, _ = _oracle_case(600, 127, 77, False)
    c4, _ = _run(x, 127, path=path, return_T=False)
    e = _err(c4, c_ref, _m4_origin(x))
    print("rel err c4 %.3e" % e)
    assert e < TOL[path]


@pytest.mark.parametrize("path", PATHS)
def test_gaussian_near_zero_cumulant(path):
    """i.i.d. Gaussian: c4 is sampling noise around zero while m4 is not."""
    x = synth.iid_gauss(40000, 43).astype(np.float32)
    c4, _ = _run(x, 24, path=path, return_T=False)
    e = _err(c4, oracle.c4_support(x, 24), _m4_origin(x))
    print("rel err c4 %.3e" % e)
    assert e < TOL[path]


def test_float64_input_and_dft_sizes():
    x = synth.cubic_process(2500, 5)
    for nfft in (40, 45, 54):   # >= 2M with the Parzen window
        c4, T = _run(x, 20, nfft)
        c_ref, T_ref = oracle.trispectrum(x, 20, nfft)
        assert _err(c4, c_ref, _m4_origin(x)) < 1e-6
        assert _err(T, T_ref, np.max(np.abs(T_ref))) < 1e-6, nfft


@pytest.mark.parametrize("window", ["none", "separable"])
def test_windows_beyond_the_support_are_refused(window):
    """The separable window and no window are nonzero where the span
    exceeds M (up to 2M), outside the contraction's lags: HOS_EUNSUPPORTED."""
    hos = pytest.importorskip("paper_1805_11775_amd")
    x = torch.from_numpy(synth.cubic_process(2500, 5)).cuda()
    with pytest.raises(hos.HosError) as e:
        hos.trispectrum(x, 20, 41 + 4, window=window)
    assert e.value.status == hos.HOS_EUNSUPPORTED


def test_impulse_uncentered_closed_form():
    """x = A delta_{t0}, no mean removal: m4 = A^4/n at the origin only,
    c2 = A^2/n at lag 0 only, so c4 = A^4/n [t = 0] - (A^2/n)^2 times the
    number of the three pairings {t1=0, t2=t3}, {t2=0, t1=t3}, {t3=0, t1=t2}
    that hold."""
    n, M, A = 3000, 12, 2.0
    x = np.zeros(n)
    x[1500] = A
    c4, _ = _run(x, M, center=False, return_T=False)
    t = np.arange(-M, M + 1)
    t1, t2, t3 = np.meshgrid(t, t, t, indexing="ij")
    pairs = ((t1 == 0) & (t2 == t3)).astype(float) + ((t2 == 0) & (t1 == t3)) + \
        ((t3 == 0) & (t1 == t2))
    expect = A ** 4 / n * ((t1 == 0) & (t2 == 0) & (t3 == 0)) - (A * A / n) ** 2 * pairs
    expect[oracle.span4(M) > M] = 0.0
    assert np.max(np.abs(c4 - expect)) < 1e-6 * A ** 4 / n


def test_constant_series_is_zero():
    c4, T = _run(np.full(2000, -1.25), 10, 20)
    assert np.max(np.abs(c4)) == 0.0 and np.max(np.abs(T)) == 0.0


def test_deterministic_and_workspace_independent():
    hos = _hos()
    x = torch.from_numpy(synth.cubic_process(100000, 9).astype(np.float32)).cuda()
    M, nfft = 40, 80
    c4a, Ta = hos.trispectrum(x, M, nfft=nfft, path="split_fp16")
    nb = hos.hos_trispectrum_workspace(x.numel(), M, nfft, hos.HOS_PATH_SPLIT_FP16)
    ws = torch.full((nb,), 0xFF, dtype=torch.uint8, device="cuda")  # NaN bytes
    c4b, Tb = hos.trispectrum(x, M, nfft=nfft, path="split_fp16", workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(c4a, c4b) and torch.equal(Ta, Tb)
    assert not torch.isnan(c4a).any()


@pytest.mark.parametrize("path", PATHS)
def test_workload_sampled(path):
    """n = 2^18 float32 cubic process, M = 48, 96^3 DFT (the benchmark shape
    and launch configuration): sampled lags against the oracle, the 24-fold
    lag symmetry and the spectrum symmetries everywhere, sampled frequencies
    against a direct sum over the returned c4."""
    x, cfg = synth.workload_trispectrum()
    M, N = cfg["M"], cfg["nfft"]
    c4, T = _run(x, M, N, path=path)
    rng = np.random.default_rng(6)
    t = rng.integers(-M, M + 1, (300, 3))
    orbit = np.array([[1, 2, 3], [3, 2, 1], [-1, 1, 2], [-3, -2, -1], [0, 0, 0],
                      [M, 0, 0], [0, M, M], [M, M, M], [-M, -M, 0], [32, 32, 31],
                      [0, 32, 48], [1, 1, 0]])
    t = np.concatenate([t, orbit])
    ref = oracle.c4_at(x, t[:, 0], t[:, 1], t[:, 2])
    span = np.maximum(t.max(1), 0) - np.minimum(t.min(1), 0)
    ref[span > M] = 0.0
    got = c4[t[:, 0] + M, t[:, 1] + M, t[:, 2] + M]
    e = float(np.max(np.abs(got - ref)) / _m4_origin(x))
    print("sampled rel err c4 %.3e (vs max|c4| %.3e)" %
          (e, np.max(np.abs(got - ref)) / np.max(np.abs(c4))))
    assert e < TOL[path]
    # one table entry per orbit: the 24 relabellings agree exactly
    for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0), (1, 2, 0)]:
        assert np.array_equal(c4, c4.transpose(perm))
    i = np.arange(2 * M + 1)
    # shift by -t1: c4(t1,t2,t3) = c4(-t1, t2-t1, t3-t1) where all lie in range
    a, b, c = np.meshgrid(i - M, i - M, i - M, indexing="ij")
    ok = (np.abs(b - a) <= M) & (np.abs(c - a) <= M)
    assert np.array_equal(c4[ok], c4[(-a)[ok] + M, (b - a)[ok] + M, (c - a)[ok] + M])
    # spectrum: Hermitian and symmetric under permutations of (k1, k2, k3)
    k = np.arange(N)
    tol = 1e-9 * np.max(np.abs(T))
    Tm = T[(-k[:, None, None]) % N, (-k[None, :, None]) % N, (-k[None, None, :]) % N]
    assert np.max(np.abs(T - np.conj(Tm))) < tol
    assert np.max(np.abs(T - T.transpose(1, 0, 2))) < tol
    assert np.max(np.abs(T - T.transpose(0, 2, 1))) < tol
    # the DFT stage at sampled frequencies
    cw = c4 * oracle.window4(M)
    lag = np.arange(-M, M + 1)
    for k1, k2, k3 in [(0, 0, 0), (1, 2, 3), (17, 40, 5), (47, 48, 95), (95, 1, 60)]:
        ph = np.exp(-2j * np.pi * (k1 * lag[:, None, None] + k2 * lag[None, :, None] +
                                   k3 * lag[None, None, :]) / N)
        assert abs(np.sum(cw * ph) - T[k1, k2, k3]) < 1e-10 * np.max(np.abs(T))


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_max_dft(path):
    """N = 512, the largest trispectrum DFT (2.1 GB), at M = 127 (n = 900):
    c4 at sampled lags against the oracle's sums, and the spectrum's
    symmetries -- Hermitian, and invariant under permutations of
    (k1, k2, k3) -- at sampled points."""
    hos = _hos()
    M, N, n = 127, 512, 900
    x = synth.cubic_process(n, 94).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    print("case: trispectrum max dft n=%d M=%d N=%d path=%s" % (n, M, N, path), flush=True)
    c4, T = hos.trispectrum(t, M, nfft=N, path=path)
    torch.cuda.synchronize()
    rng = np.random.default_rng(15)
    w = rng.integers(-M, M + 1, (400, 3))
    lo = np.minimum(0, w.min(1)); hi = np.maximum(0, w.max(1))
    w = w[hi - lo <= M]
    w = np.concatenate([w, [[0, 0, 0], [1, 2, 3], [M, M, 0]]])
    ref = oracle.c4_at(x, w[:, 0], w[:, 1], w[:, 2])
    idx = [torch.from_numpy(w[:, j] + M).cuda() for j in range(3)]
    got = c4[idx[0], idx[1], idx[2]].cpu().numpy()
    e = _err(got, ref, _m4_origin(x))
    print("sampled err c4 %.3e" % e)
    assert e < TOL[path]
    k = torch.from_numpy(rng.integers(0, N, (4000, 3))).cuda()
    q = T[k[:, 0], k[:, 1], k[:, 2]]
    qp = T[k[:, 2], k[:, 0], k[:, 1]]
    qc = T[(-k[:, 0]) % N, (-k[:, 1]) % N, (-k[:, 2]) % N].conj()
    scale = float(T.abs().max())
    s1 = float((q - qp).abs().max()) / scale
    s2 = float((q - qc).abs().max()) / scale
    print("symmetry %.3e %.3e" % (s1, s2))
    assert s1 < 1e-12 and s2 < 1e-12


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_spectrum_alone_equals_spectrum_with_cumulant(path):
    """Asking for T alone folds the c4 cube from the workspace instead of the
    caller's c4 array: the same kernels on the same data, so T must equal
    the T of the call that also returns c4, bit for bit."""
    hos = _hos()
    x = synth.cubic_process(3000, 83).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    print("case: T alone n=3000 M=20 N=48 path=%s" % path, flush=True)
    _, T_both = hos.trispectrum(t, 20, nfft=48, path=path)
    c4_none, T_only = hos.trispectrum(t, 20, nfft=48, path=path, return_c4=False)
    torch.cuda.synchronize()
    assert c4_none is None
    assert torch.equal(T_only, T_both)
