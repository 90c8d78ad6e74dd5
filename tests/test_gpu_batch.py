"""GPU parity of the batched bispectra and of the loss and its adjoint
against the FP64 oracle (per-series definitions).

Bars as for one series: normwise 1e-6 (FP32 path) and 1e-5 (split paths)
for c3 (over each series' hexagon) and B (over its principal domain); the
same bars for the gradient, normwise over each series.
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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) /
                 max(np.max(np.abs(np.asarray(b))), 1e-300))


def _uneven():
    spec = [(700, 0), (701, 5), (3001, 31), (2500, 64), (1800, 96), (4100, 128), (2200, 200),
            (1537, 33)]
    xs = []
    for k, (n, M) in enumerate(spec):
        x = synth.iid_gauss(n, 50 + k) if k % 2 == 0 else synth.iid_exp_centered(n, 50 + k)
        xs.append(x.astype(np.float32))
    return xs, [n for n, _ in spec], [M for _, M in spec]


@pytest.mark.parametrize("path", PATHS)
def test_uneven_batch_matches_oracle(path):
    hos = _hos()
    xs, n, M = _uneven()
    plan = hos.BatchPlan(n, M, path=path)
    print("case: uneven batch of %d, path %s, items %s" %
          (len(n), path, (plan.info["items0"], plan.info["items1"])), flush=True)
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    c3, B = hos.bispectrum_batched(x, plan)
    torch.cuda.synchronize()
    c3, B = c3.cpu().numpy(), B.cpu().numpy()
    S = plan.series()
    for s in range(len(n)):
        Ms, N, npd, c3o, pdo = int(S[s, 1]), int(S[s, 2]), int(S[s, 3]), int(S[s, 5]), int(S[s, 6])
        c_ref, B_ref = oracle.bispectrum(xs[s], Ms, N)
        k1, k2 = oracle.pd_indices(N)
        got_c = c3[c3o:c3o + (2 * Ms + 1) ** 2].reshape(2 * Ms + 1, 2 * Ms + 1)
        e1, e2 = _rel(got_c, c_ref), _rel(B[pdo:pdo + npd], B_ref[k1, k2])
        print("series %d n=%d M=%d: c3 %.3e B_pd %.3e" % (s, n[s], Ms, e1, e2))
        assert e1 < TOL[path] and e2 < TOL[path], (s, e1, e2)


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_batch_spectra_each_dft_size(path):
    """One short series per DFT size of the batch spectra's fixed-size
    kernels (N = 64, 128, 256, 512, 1024) and one size they leave to the
    general kernels (N = 200): c3 and the principal-domain spectrum of every
    series against the oracle, element by element."""
    hos = _hos()
    M = [32, 64, 128, 256, 512, 100]
    n = [1300, 1400, 1500, 1600, 1700, 1250]
    xs = [(synth.iid_gauss(k, 90 + i) if i % 2 == 0 else synth.iid_exp_centered(k, 90 + i))
          .astype(np.float32) for i, k in enumerate(n)]
    plan = hos.BatchPlan(n, M, path=path)
    S = plan.series()
    assert [int(v) for v in S[:, 2]] == [64, 128, 256, 512, 1024, 200]
    print("case: batch spectra sizes, path %s" % path, flush=True)
    c3, B = hos.bispectrum_batched(torch.from_numpy(np.concatenate(xs)).cuda(), plan)
    torch.cuda.synchronize()
    c3, B = c3.cpu().numpy(), B.cpu().numpy()
    for s in range(len(n)):
        Ms, N, npd, c3o, pdo = int(S[s, 1]), int(S[s, 2]), int(S[s, 3]), int(S[s, 5]), int(S[s, 6])
        c_ref, B_ref = oracle.bispectrum(xs[s], Ms, N)
        k1, k2 = oracle.pd_indices(N)
        got_c = c3[c3o:c3o + (2 * Ms + 1) ** 2].reshape(2 * Ms + 1, 2 * Ms + 1)
        e1, e2 = _rel(got_c, c_ref), _rel(B[pdo:pdo + npd], B_ref[k1, k2])
        print("series %d n=%d M=%d N=%d: c3 %.3e B_pd %.3e" % (s, n[s], Ms, N, e1, e2))
        assert e1 < TOL[path] and e2 < TOL[path], (s, e1, e2)


def test_batch_deterministic():
    hos = _hos()
    xs, n, M = _uneven()
    plan = hos.BatchPlan(n, M, path="split_fp16")
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    a = hos.bispectrum_batched(x, plan)
    b = hos.bispectrum_batched(x, plan)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_workload_batch_sampled():
    """4096 float32 series, n in [1024, 65536], M in {32, 64, 128, 256}
    (the batched benchmark shape and plan: the tiles of the shipped tuned
    table, one launch over both tile classes): c3 at sampled lags of a
    stratified subset against the oracle, the principal-domain spectra of two
    series in full."""
    hos = _hos()
    from paper_1805_11775_amd import tune
    xs, n, M = synth.workload_batched()
    table = tune.load(tune.device_key("split_fp16"))
    assert table is not None, "no shipped tile table for this device"
    plan = hos.BatchPlan(n, M, path="split_fp16", tile=tune.tiles_for(n, M, table))
    print("case: batch of %d, ws %.1f GB, items %s" %
          (len(n), plan.info["ws_bytes"] / 1e9, (plan.info["items0"], plan.info["items1"])),
          flush=True)
    x = torch.from_numpy(np.concatenate(xs).astype(np.float32)).cuda()
    c3, B = hos.bispectrum_batched(x, plan)
    torch.cuda.synchronize()
    S = plan.series()
    # stratified: each M with each distribution, and the shortest / longest
    pick = set()
    for m in (32, 64, 128, 256):
        for par in (0, 1):
            idx = [k for k in range(len(n)) if M[k] == m and k % 2 == par]
            pick.add(idx[0])
    pick.add(int(np.argmin(n)))
    pick.add(int(np.argmax(n)))
    rng = np.random.default_rng(8)
    for s in sorted(pick):
        Ms, c3o = int(S[s, 1]), int(S[s, 5])
        xs32 = xs[s].astype(np.float32)
        side = 2 * Ms + 1
        got = c3[c3o:c3o + side * side].view(side, side).cpu().numpy()
        w1 = rng.integers(-Ms, Ms + 1, 60)
        w2 = np.clip(w1 + rng.integers(-Ms, Ms + 1, 60), -Ms, Ms)
        w1 = np.concatenate([w1, [0, 1, Ms]])
        w2 = np.concatenate([w2, [0, 2, 0]])
        ref = oracle.c3_at(xs32, w1, w2)
        ref[np.abs(w1 - w2) > Ms] = 0.0
        e = np.max(np.abs(got[w1 + Ms, w2 + Ms] - ref)) / np.max(np.abs(ref))
        print("series %d n=%d M=%d sampled c3 %.3e" % (s, n[s], Ms, e))
        assert e < 1e-5
    for s in (int(np.argmin(n)), [k for k in range(len(n)) if M[k] == 64][0]):
        Ms, N, npd, pdo = int(S[s, 1]), int(S[s, 2]), int(S[s, 3]), int(S[s, 6])
        _, B_ref = oracle.bispectrum(xs[s].astype(np.float32), Ms, N)
        k1, k2 = oracle.pd_indices(N)
        e = _rel(B[pdo:pdo + npd].cpu().numpy(), B_ref[k1, k2])
        print("series %d B_pd %.3e" % (s, e))
        assert e < 1e-5


def _loss_setup(path, batch=3, n=3000, M=20, N=40):
    hos = _hos()
    X = np.stack([synth.iid_gauss(n, 70 + b) for b in range(batch)]).astype(np.float32)
    tgt = synth.quadratic_process(n, 99).astype(np.float32)
    k1, k2 = oracle.pd_indices(N)
    target = oracle.bispectrum(tgt, M, N)[1][k1, k2]
    plan = hos.BatchPlan([n] * batch, [M] * batch, path=path, adjoint=True)
    return hos, X, target, plan


@pytest.mark.parametrize("path", PATHS)
def test_loss_forward(path):
    hos, X, target, plan = _loss_setup(path)
    print("case: loss forward, path %s" % path, flush=True)
    x = torch.from_numpy(X).cuda()
    loss, B = hos.bispectrum_loss_fwd(x, torch.from_numpy(target), plan)
    torch.cuda.synchronize()
    ref = oracle.bispectrum_loss(X, 20, 40, target)
    e = abs(float(loss) - ref) / ref
    print("loss rel err %.3e" % e)
    assert e < TOL[path]


@pytest.mark.parametrize("path", PATHS)
def test_loss_gradient(path):
    """The adjoint against the oracle's gradient (itself pinned by central
    differences), and through torch.autograd with an upstream scale."""
    hos, X, target, plan = _loss_setup(path)
    print("case: loss gradient, path %s" % path, flush=True)
    x = torch.from_numpy(X).cuda().requires_grad_(True)
    loss = hos.bispectrum_loss(x, torch.from_numpy(target).cuda(), plan)
    (g,) = torch.autograd.grad(2.5 * loss, x)
    torch.cuda.synchronize()
    ref = oracle.bispectrum_loss_grad(X, 20, 40, target, dL=2.5)
    g = g.cpu().numpy()
    for b in range(X.shape[0]):
        e = _rel(g[b], ref[b])
        print("series %d grad rel err %.3e" % (b, e))
        assert e < TOL[path]


def test_loss_gradient_float64():
    hos = _hos()
    n, M, N = 1500, 12, 24
    X = np.stack([synth.iid_exp_centered(n, 80 + b) for b in range(2)])
    tgt = synth.quadratic_process(n, 98)
    k1, k2 = oracle.pd_indices(N)
    target = oracle.bispectrum(tgt, M, N)[1][k1, k2]
    plan = hos.BatchPlan([n, n], [M, M], path="fp32", adjoint=True)
    x = torch.from_numpy(X).cuda()
    loss, B = hos.bispectrum_loss_fwd(x, torch.from_numpy(target), plan)
    dx = hos.bispectrum_loss_bwd(x, torch.from_numpy(target), B,
                                 torch.ones((), dtype=torch.float64), plan)
    torch.cuda.synchronize()
    assert abs(float(loss) - oracle.bispectrum_loss(X, M, N, target)) < 1e-6 * float(loss)
    ref = oracle.bispectrum_loss_grad(X, M, N, target)
    assert _rel(dx.cpu().numpy(), ref) < 1e-6


@pytest.mark.parametrize("M", [7, 11])
def test_loss_gradient_dft_sizes_above_2M(M):
    """DFT sizes other than 2M: M = 7 takes N = 15 (odd: one lag per grid
    row), M = 11 takes N = 24 (row 12 holds no lag of [-M, M]); the lag
    weights come straight from the residual's row transforms either way."""
    hos = _hos()
    n = 1800
    N = hos.default_nfft(M)
    assert N > 2 * M
    X = np.stack([synth.iid_exp_centered(n, 60 + M + b) for b in range(2)]).astype(np.float32)
    tgt = synth.quadratic_process(n, 61)
    k1, k2 = oracle.pd_indices(N)
    target = oracle.bispectrum(tgt, M, N)[1][k1, k2]
    plan = hos.BatchPlan([n, n], [M, M], path="split_fp16", adjoint=True)
    assert (plan.series()[:, 2] == N).all()
    print("case: loss gradient M=%d N=%d" % (M, N), flush=True)
    x = torch.from_numpy(X).cuda()
    loss, B = hos.bispectrum_loss_fwd(x, torch.from_numpy(target), plan)
    dx = hos.bispectrum_loss_bwd(x, torch.from_numpy(target), B,
                                 torch.ones((), dtype=torch.float64), plan)
    torch.cuda.synchronize()
    ref = oracle.bispectrum_loss_grad(X, M, N, target)
    dx = dx.cpu().numpy()
    for b in range(2):
        e = _rel(dx[b], ref[b])
        print("series %d grad rel err %.3e" % (b, e))
        assert e < TOL["split_fp16"]


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_loss_gradient_largest_lag(path):
    """The adjoint at the largest lag it takes (M = 320, N = 640: the
    largest staged window, several 1024-row workgroups of the contraction,
    series of uneven length with partial last workgroups) against the
    oracle's full gradient."""
    hos = _hos()
    n, M, N = [2600, 1900], 320, 640
    X = [synth.iid_exp_centered(k, 90 + i).astype(np.float32) for i, k in enumerate(n)]
    tgt = synth.quadratic_process(2400, 97)
    k1, k2 = oracle.pd_indices(N)
    target = oracle.bispectrum(tgt, M, N)[1][k1, k2]
    plan = hos.BatchPlan(n, [M, M], path=path, adjoint=True)
    print("case: loss gradient M=320, path %s" % path, flush=True)
    x = torch.from_numpy(np.concatenate(X)).cuda()
    loss, B = hos.bispectrum_loss_fwd(x, torch.from_numpy(target), plan)
    dx = hos.bispectrum_loss_bwd(x, torch.from_numpy(target), B,
                                 torch.ones((), dtype=torch.float64), plan)
    torch.cuda.synchronize()
    dx = dx.cpu().numpy()
    off = 0
    for b, xb in enumerate(X):
        ref = oracle.bispectrum_loss_grad(xb, M, N, target)
        e = _rel(dx[off:off + xb.size], ref)
        print("series %d grad rel err %.3e" % (b, e))
        assert e < TOL[path]
        off += xb.size


@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_loss_workload_sampled(path):
    """64 float32 N(0,1) series of n = 65536, M = 256, N = 512 (the
    differentiable-bispectrum shape): loss of two series and gradient
    differences at sampled samples against the oracle; the gradient sums to
    zero per series."""
    hos = _hos()
    X, tgt, cfg = synth.workload_loss()
    M, N = cfg["M"], cfg["nfft"]
    k1, k2 = oracle.pd_indices(N)
    plan = hos.BatchPlan([X.shape[1]] * X.shape[0], [M] * X.shape[0], path=path, adjoint=True)
    print("case: loss workload, path %s, ws %.2f GB" % (path, plan.info["ws_bytes"] / 1e9),
          flush=True)
    _, Bt = hos.bispectrum_batched(torch.from_numpy(tgt.astype(np.float32)).cuda(),
                                   hos.BatchPlan([tgt.size], [M], path="fp32"), return_c3=False)
    target = Bt
    x = torch.from_numpy(X).cuda()
    loss, B = hos.bispectrum_loss_fwd(x, target, plan)
    dx = hos.bispectrum_loss_bwd(x, target, B, torch.ones((), dtype=torch.float64), plan)
    torch.cuda.synchronize()
    tnp = target.cpu().numpy()
    Bn = B.cpu().numpy().reshape(X.shape[0], -1)
    dxn = dx.cpu().numpy().reshape(X.shape)
    rng = np.random.default_rng(4)
    for b in (37,):
        Bref = oracle.bispectrum_pd(X[b], M, N)
        e = _rel(Bn[b], Bref)
        print("series %d B_pd %.3e" % (b, e))
        assert e < TOL[path]
        idx = np.concatenate([[0, 1, 255, 256, 65535], rng.integers(0, X.shape[1], 40)])
        ga = oracle.loss_grad_at(X[b], M, N, tnp, idx)
        d_ref = ga[1:] - ga[0]
        d_got = dxn[b, idx[1:]] - dxn[b, idx[0]]
        e = np.max(np.abs(d_got - d_ref)) / np.max(np.abs(ga))
        print("series %d sampled grad %.3e" % (b, e))
        assert e < TOL[path]
        assert abs(np.sum(dxn[b].astype(np.float64))) < 1e-3 * np.max(np.abs(dxn[b])) * 256
    assert np.isfinite(float(loss))


def test_tuner_choices_are_valid_and_correct(tmp_path):
    """hos_tune through the tuner: one tile choice per (lag, length bucket)
    among the candidates with its timings, merged into a cache under the
    device's key and read back; a plan built from the choices matches the
    oracle."""
    hos = _hos()
    from paper_1805_11775_amd import tune
    cache = str(tmp_path / "tiles.json")
    res = tune.tune([32, 128], path="split_fp16", edges=(1024, 2048, 8192), series=6, reps=2,
                    cache=cache)
    print("tuned:", res, flush=True)
    assert set(res["choices"]) == {32, 128}
    assert all(v in (2, 4) for row in res["choices"].values() for v in row)
    assert all(len(row) == 2 for row in res["choices"].values())
    assert all(t > 0 for row in res["ms"].values() for pair in row for t in pair)
    table = tune.load(tune.device_key("split_fp16"), cache)
    assert table["choices"] == res["choices"] and table["edges"] == [1024, 2048, 8192]
    xs = [synth.iid_exp_centered(3000, 91).astype(np.float32),
          synth.iid_gauss(2500, 92).astype(np.float32)]
    tiles = tune.tiles_for([3000, 2500], [32, 128], table)
    assert tiles == [res["choices"][32][1], res["choices"][128][1]]
    plan = hos.BatchPlan([3000, 2500], [32, 128], path="split_fp16", tile=tiles)
    c3, B = hos.bispectrum_batched(torch.from_numpy(np.concatenate(xs)).cuda(), plan)
    torch.cuda.synchronize()
    S = plan.series()
    for s in range(2):
        Ms, N, npd, c3o, pdo = (int(v) for v in (S[s, 1], S[s, 2], S[s, 3], S[s, 5], S[s, 6]))
        c_ref, B_ref = oracle.bispectrum(xs[s], Ms, N)
        k1, k2 = oracle.pd_indices(N)
        got = c3[c3o:c3o + (2 * Ms + 1) ** 2].cpu().numpy().reshape(2 * Ms + 1, -1)
        assert _rel(got, c_ref) < 1e-5
        assert _rel(B[pdo:pdo + npd].cpu().numpy(), B_ref[k1, k2]) < 1e-5


@pytest.mark.parametrize("tile", [2, 4])
def test_forced_tile_classes_match_oracle(tile):
    """Every series on one tile class, whatever its lag."""
    hos = _hos()
    xs, n, M = _uneven()
    plan = hos.BatchPlan(n, M, path="split_fp16", tile=[tile] * len(n))
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    c3, B = hos.bispectrum_batched(x, plan)
    torch.cuda.synchronize()
    c3, B = c3.cpu().numpy(), B.cpu().numpy()
    S = plan.series()
    for s in range(len(n)):
        Ms, N, npd, c3o, pdo = (int(v) for v in (S[s, 1], S[s, 2], S[s, 3], S[s, 5], S[s, 6]))
        c_ref, B_ref = oracle.bispectrum(xs[s], Ms, N)
        k1, k2 = oracle.pd_indices(N)
        got = c3[c3o:c3o + (2 * Ms + 1) ** 2].reshape(2 * Ms + 1, 2 * Ms + 1)
        assert _rel(got, c_ref) < 1e-5 and _rel(B[pdo:pdo + npd], B_ref[k1, k2]) < 1e-5, s




@pytest.mark.parametrize("path", ["split_fp16", "fp32"])
def test_max_lag_in_batch(path):
    """M = 1024 (N = 2048, the largest DFT of a batch) beside two small
    series: c3 and the principal-domain spectrum of every series against
    the oracle."""
    hos = _hos()
    n = [4000, 1500, 2100]
    M = [1024, 32, 7]
    xs = [synth.iid_exp_centered(k, 60 + i).astype(np.float32) for i, k in enumerate(n)]
    plan = hos.BatchPlan(n, M, path=path)
    print("case: batch with M=1024, path %s" % path, flush=True)
    c3, B = hos.bispectrum_batched(torch.from_numpy(np.concatenate(xs)).cuda(), plan)
    torch.cuda.synchronize()
    c3, B = c3.cpu().numpy(), B.cpu().numpy()
    S = plan.series()
    for s in range(len(n)):
        Ms, N, npd, c3o, pdo = int(S[s, 1]), int(S[s, 2]), int(S[s, 3]), int(S[s, 5]), int(S[s, 6])
        c_ref, B_ref = oracle.bispectrum(xs[s], Ms, N)
        k1, k2 = oracle.pd_indices(N)
        got_c = c3[c3o:c3o + (2 * Ms + 1) ** 2].reshape(2 * Ms + 1, 2 * Ms + 1)
        e1, e2 = _rel(got_c, c_ref), _rel(B[pdo:pdo + npd], B_ref[k1, k2])
        print("series %d n=%d M=%d N=%d: c3 %.3e B_pd %.3e" % (s, n[s], Ms, N, e1, e2))
        assert e1 < TOL[path] and e2 < TOL[path], (s, e1, e2)
