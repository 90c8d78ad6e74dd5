"""GPU parity of the order-five path against the FP64 oracle.

Error measure for c5: max|GPU - oracle| over the hypercube divided by the
fifth absolute moment (1/n) sum |x~|^5, which bounds |m5| at every lag
(Hoelder) -- the contraction that forms m5 is the only reduced-precision
step; c2 and c3 are FP64 on every path.  The spectrum is measured against
the bound the same scale puts on it, |Q| <= (1/n) sum |x~|^5 * sum_t W5(t):
c5 is a small difference of moments (m5 minus ten c2 c3 products), so
max|Q| itself can sit orders of magnitude below the scale of the rounding.
Bars: 1e-6 (FP32 path), 1e-5 (split paths)."""
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


def _run(x, M, nfft=None, **kw):
    hos = _hos()
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    print("case: n=%d M=%d nfft=%s %s dtype=%s" % (t.numel(), M, nfft, kw, t.dtype), flush=True)
    c5, Q = hos.cumulant5(t, M, nfft=nfft, **kw)
    torch.cuda.synchronize()
    return (c5.cpu().numpy() if c5 is not None else None,
            Q.cpu().numpy() if Q is not None else None)


def _scale(x, center=True):
    xt = x - np.mean(x) if center else np.asarray(x, dtype=np.float64)
    return float(np.mean(np.abs(xt) ** 5))


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,M", [(1500, 0), (1500, 1), (2001, 4), (1800, 8), (1200, 10)])
def test_parity_hypercube(path, n, M):
    x = synth.quartic_process(n, 300 + n + M).astype(np.float32)
    N = _hos().default_nfft(M)
    c5, Q = _run(x, M, N, path=path)
    c_ref, Q_ref = oracle.spectrum5(x, M, N)
    e1 = float(np.max(np.abs(c5 - c_ref)) / _scale(x))
    e2 = float(np.max(np.abs(Q - Q_ref)) / (_scale(x) * np.sum(oracle.window5(M))))
    print("rel err c5 %.3e Q %.3e" % (e1, e2))
    assert e1 < TOL[path] and e2 < TOL[path]


@pytest.mark.parametrize("window", ["none", "separable"])
def test_windows_beyond_the_support_are_refused(window):
    """Only the Parzen product over every pairwise difference vanishes
    where the span exceeds M; the other windows would need c5 there, which
    the contraction does not compute: HOS_EUNSUPPORTED, nothing launched."""
    hos = _hos()
    x = torch.from_numpy(synth.iid_exp_centered(1600, 12)).cuda()
    M = 5
    N = hos.default_nfft(M, window)
    with pytest.raises(hos.HosError) as e:
        hos.cumulant5(x, M, N, window=window, path="fp32")
    assert e.value.status == hos.HOS_EUNSUPPORTED


def test_uncentred_impulse_closed_form():
    """x = A delta, no mean removal: A^5/n at the origin minus (A^2/n)(A^3/n)
    times the number of pair / triple splits whose blocks are each constant
    (the oracle pin's closed form), on the GPU path in float64."""
    n, A, M = 2000, 1.5, 3
    x = np.zeros(n)
    x[1000] = A
    c5, _ = _run(x, M, center=False, return_Q=False, path="fp32")
    t = np.arange(-M, M + 1)
    g = np.meshgrid(t, t, t, t, indexing="ij")
    pts = [np.zeros_like(g[0])] + list(g)
    count = np.zeros_like(g[0], dtype=float)
    for j in range(5):
        for k in range(j + 1, 5):
            rest = [pts[i] for i in range(5) if i not in (j, k)]
            count += ((pts[j] == pts[k]) & (rest[0] == rest[1]) & (rest[1] == rest[2]))
    alleq = (g[0] == 0) & (g[1] == 0) & (g[2] == 0) & (g[3] == 0)
    expect = A ** 5 / n * alleq - (A ** 2 / n) * (A ** 3 / n) * count
    expect[oracle.span5(M) > M] = 0.0
    assert np.max(np.abs(c5 - expect)) < 1e-6 * A ** 5 / n


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_workload_sampled(path):
    """n = 2^18 float32 quartic process, M = 24, 48^4 DFT (the benchmark
    shape): sampled lags against the oracle, the 120-fold symmetry exactly,
    and sampled frequencies against a direct sum over the returned c5."""
    x, cfg = synth.workload_cumulant5()
    M, N = cfg["M"], cfg["nfft"]
    c5, Q = _run(x, M, N, path=path)
    rng = np.random.default_rng(3)
    t = rng.integers(-M, M + 1, (200, 4))
    t = np.concatenate([t, [[-1, -2, -3, -4], [1, 2, 3, 4], [0, 0, 0, 0], [M, 0, 0, 0],
                            [24, 24, 23, 1]]])
    span = np.maximum(t.max(1), 0) - np.minimum(t.min(1), 0)
    ref = oracle.c5_at(x, t[:, 0], t[:, 1], t[:, 2], t[:, 3])
    ref[span > M] = 0.0
    got = c5[t[:, 0] + M, t[:, 1] + M, t[:, 2] + M, t[:, 3] + M]
    e = float(np.max(np.abs(got - ref)) / _scale(x))
    print("sampled rel err c5 %.3e; c5 at the orbit of (1,2,3,4): %.4f" %
          (e, c5[M + 1, M + 2, M + 3, M + 4]))
    assert e < TOL[path]
    for perm in [(1, 0, 2, 3), (0, 2, 3, 1), (3, 2, 1, 0)]:
        assert np.array_equal(c5, c5.transpose(perm))
    cw = c5 * oracle.window5(M)
    lag = np.arange(-M, M + 1)
    for k in [(0, 0, 0, 0), (1, 2, 3, 4), (47, 5, 20, 33)]:
        ph = np.exp(-2j * np.pi * (k[0] * lag[:, None, None, None] +
                                   k[1] * lag[None, :, None, None] +
                                   k[2] * lag[None, None, :, None] +
                                   k[3] * lag[None, None, None, :]) / N)
        assert abs(np.sum(cw * ph) - Q[k]) < 1e-9 * np.max(np.abs(Q))


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_max_lag_and_dft(path):
    """M = 40 and N = 96, the largest lag and DFT of order five (n = 3000):
    c5 at sampled lags against the oracle's sums (error against the fifth
    absolute moment, as above), and the spectrum's symmetries: Q is
    Hermitian and invariant under permutations of (k1..k4), at sampled
    points."""
    hos = _hos()
    M, N, n = 40, 96, 3000
    x = synth.quartic_process(n, 93).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    print("case: order five max n=%d M=%d N=%d path=%s" % (n, M, N, path), flush=True)
    c5, Q = hos.cumulant5(t, M, nfft=N, path=path)
    torch.cuda.synchronize()
    rng = np.random.default_rng(14)
    w = rng.integers(-M, M + 1, (400, 4))
    lo = np.minimum(0, w.min(1)); hi = np.maximum(0, w.max(1))
    w = w[hi - lo <= M]
    w = np.concatenate([w, [[0, 0, 0, 0], [1, 2, 3, 4], [M, M, 0, M]]])
    ref = oracle.c5_at(x, w[:, 0], w[:, 1], w[:, 2], w[:, 3])
    idx = [torch.from_numpy(w[:, j] + M).cuda() for j in range(4)]
    got = c5[idx[0], idx[1], idx[2], idx[3]].cpu().numpy()
    e = float(np.max(np.abs(got - ref))) / _scale(x)
    print("sampled err c5 %.3e" % e)
    assert e < TOL[path]
    k = torch.from_numpy(rng.integers(0, N, (4000, 4))).cuda()
    q = Q[k[:, 0], k[:, 1], k[:, 2], k[:, 3]]
    qp = Q[k[:, 2], k[:, 0], k[:, 3], k[:, 1]]
    qc = Q[(-k[:, 0]) % N, (-k[:, 1]) % N, (-k[:, 2]) % N, (-k[:, 3]) % N].conj()
    scale = float(Q.abs().max())
    s1 = float((q - qp).abs().max()) / scale
    s2 = float((q - qc).abs().max()) / scale
    print("symmetry %.3e %.3e" % (s1, s2))
    assert s1 < 1e-12 and s2 < 1e-12


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_spectrum_alone_equals_spectrum_with_cumulant(path):
    """Asking for Q alone folds the cumulant cube from the workspace instead
    of the caller's c5 array: the same kernels on the same data, so Q must
    equal the Q of the call that also returns c5, bit for bit."""
    x = synth.quartic_process(2500, 71).astype(np.float32)
    _, Q_both = _run(x, 12, 32, path=path)
    c5_none, Q_only = _run(x, 12, 32, path=path, return_c5=False)
    assert c5_none is None
    assert np.array_equal(Q_only, Q_both)
