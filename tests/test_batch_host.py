"""Host-side checks of batch plans: work items cover every (series, tile,
chunk) once, slots are consistent, the LPT assignment is balanced, series
offsets and DFT sizes follow the documented packing, and the batched entry
points reject bad arguments before touching a device."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1805_11775_amd as hos
import synth


def _fft_ok(N):
    m = N
    for r in (2, 3, 5):
        while m % r == 0:
            m //= r
    return m == 1


def _expected_N(M, window):
    k = max(2, 2 * M if window == "parzen" else 2 * M + 1)
    while not _fft_ok(k):
        k += 1
    return k


CASES = [
    ([700, 5000, 3001, 1200, 65536], [0, 5, 64, 100, 256], "split_fp16"),
    ([2048] * 8, [64] * 8, "fp32"),
    ([65536] * 64, [256] * 64, "split_fp16"),
    ([1500, 1501, 97, 4096, 513], [31, 32, 33, 96, 95], "split_bf16"),
]


@pytest.mark.parametrize("n,M,path", CASES)
def test_items_cover_every_chunk_once(n, M, path):
    plan = hos.BatchPlan(n, M, path=path)
    S = plan.series()
    for cls in (0, 1):
        NB = 4 if cls else 2
        it = plan.items(cls)
        assert len(it) == plan.info["items%d" % cls]
        seen = {}
        slots = set()
        for row in it:
            c, w, s, R, Cc, c0, c1, slot = (int(v) for v in row)
            assert c == cls and 0 <= w < plan.info["G%d" % cls] and 0 <= c0 < c1
            assert S[s, 7] == cls and 0 <= Cc <= R
            assert slot not in slots
            slots.add(slot)
            for ch in range(c0, c1):
                key = (s, R, Cc, ch)
                assert key not in seen
                seen[key] = slot
        # every tile of every series of the class, every chunk
        expect = 0
        for s in range(len(n)):
            if S[s, 7] != cls:
                continue
            nbr = (M[s] + 31) // 32
            tr = (nbr + NB - 1) // NB if nbr else 0
            # chunk length: 1024 samples on the split paths (both tile classes,
            # one launch), 512 on the FP32 path
            L = 1024 if path != "fp32" else 512
            expect += tr * (tr + 1) // 2 * ((n[s] + L - 1) // L)
        assert len(seen) == expect
        if slots:
            assert slots == set(range(len(slots)))


_MIXED = synth.batched_series(120, 4)[1:]


@pytest.mark.parametrize("n,M,path", CASES + [(list(_MIXED[0]), list(_MIXED[1]), "split_fp16")])
def test_one_launch_order(n, M, path):
    """Every item of both classes in one list: each workgroup's 4 x 4-block
    items precede its 2 x 2-block items (the kernel runs one loop per class),
    and the list is grouped by workgroup."""
    plan = hos.BatchPlan(n, M, path=path)
    it = plan.items(-1)
    assert len(it) == plan.info["items0"] + plan.info["items1"]
    assert np.all(np.diff(it[:, 1]) >= 0)
    for w in np.unique(it[:, 1]):
        cls = it[it[:, 1] == w, 0]
        assert np.all(np.diff(cls) <= 0), w   # 1 ... 1 0 ... 0


@pytest.mark.parametrize("n,M,path", CASES)
def test_lpt_balance(n, M, path):
    """One launch for both tile classes: one set of workgroups, and the
    longest-processing-time assignment over the items of both classes keeps
    every workgroup within the mean load plus one item (the greedy rule's
    bound).  Chunk costs: 14 for a 4 x 4-block tile and 5 for a 2 x 2-block
    tile on the split paths; 4 off and 3 on the diagonal on the FP32 path."""
    plan = hos.BatchPlan(n, M, path=path)
    assert plan.info["G0"] == plan.info["G1"]
    G = plan.info["G0"]
    rows = [plan.items(c) for c in (0, 1)]
    it = np.concatenate([r for r in rows if len(r)])
    cost = (it[:, 6] - it[:, 5]).astype(float)
    if path == "fp32":
        cost *= np.where(it[:, 3] == it[:, 4], 3.0, 4.0)
    else:
        cost *= np.where(it[:, 0] == 1, 14.0, 5.0)
    load = np.bincount(it[:, 1], weights=cost, minlength=G)
    assert load.max() <= load.sum() / G + cost.max() + 1e-9
    assert np.all(load > 0) and G <= 256


@pytest.mark.parametrize("window", ["none", "separable"])
def test_plan_rejects_windows_nonzero_at_the_corners(window):
    """Batches compute each series' hexagon only; the windows that do not
    vanish at the square's corners are refused before any device work."""
    n, M = synth.batched_series(8, 3)[1:]
    with pytest.raises(hos.HosError) as e:
        hos.BatchPlan(n, M, window=window, path="split_fp16")
    assert e.value.status == hos.HOS_EUNSUPPORTED


@pytest.mark.parametrize("window", ["parzen"])
def test_series_layout(window):
    n, M = synth.batched_series(40, 3)[1:]
    plan = hos.BatchPlan(n, M, window=window, path="split_fp16")
    S = plan.series()
    assert np.array_equal(S[:, 0], n) and np.array_equal(S[:, 1], M)
    assert np.array_equal(S[:, 4], np.concatenate([[0], np.cumsum(n)[:-1]]))
    side2 = (2 * np.asarray(M) + 1) ** 2
    assert np.array_equal(S[:, 5], np.concatenate([[0], np.cumsum(side2)[:-1]]))
    for s in range(len(n)):
        N = _expected_N(int(M[s]), window)
        assert S[s, 2] == N and S[s, 3] == len(oracle.pd_indices(N)[0])
    assert np.array_equal(S[:, 6], np.concatenate([[0], np.cumsum(S[:, 3])[:-1]]))
    assert plan.info["c3_elems"] == side2.sum() and plan.info["pd_elems"] == S[:, 3].sum()
    assert plan.info["x_elems"] == np.sum(n)


@pytest.mark.parametrize("n,M,kw", [
    ([100], [100], {}),                 # M >= n
    ([1], [0], {}),                     # n < 2
    ([5000], [1025], {}),               # DFT size beyond the batch limit
    ([5000], [321], {"adjoint": True}),  # beyond the adjoint's staged window
    ([100, 200], [5], {}),              # lengths differ
])
def test_plan_rejects(n, M, kw):
    with pytest.raises((hos.HosError, ValueError)):
        hos.BatchPlan(n, M, **kw)


def test_plan_rejects_enums():
    lib = hos.lib()
    n = np.array([1000], dtype=np.int64)
    M = np.array([10], dtype=np.int32)
    pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    args = (1, hos._i64p(n), hos._i32p(M))
    assert lib.hos_batch_plan_size(*args, 3, 0, 0, None, ctypes.byref(pb), ctypes.byref(wb)) == -1
    assert lib.hos_batch_plan_size(*args, 1, 3, 0, None, ctypes.byref(pb), ctypes.byref(wb)) == -1
    assert lib.hos_batch_plan_size(*args, 1, 0, 4, None, ctypes.byref(pb), ctypes.byref(wb)) == -1
    assert lib.hos_batch_plan_size(*args, 1, 0, 0, None, ctypes.byref(pb), ctypes.byref(wb)) == 0


FAKE = 0x10000


def test_batched_entry_points_validate_before_device():
    lib = hos.lib()
    plan = hos.BatchPlan([3000, 2000], [20, 20], adjoint=True)
    ph = plan.host.ctypes.data
    wsb = plan.info["ws_bytes"]
    f = lib.hos_bispectrum_batched
    assert f(FAKE, 0, ph, FAKE, FAKE, FAKE, FAKE, wsb - 1, None) == hos.HOS_EWORKSPACE
    assert f(None, 0, ph, FAKE, FAKE, FAKE, FAKE, wsb, None) == hos.HOS_EINVAL
    assert f(FAKE, 0, ph, FAKE, None, None, FAKE, wsb, None) == hos.HOS_EINVAL
    assert f(FAKE, 0, ph, FAKE + 8, FAKE, FAKE, FAKE, wsb, None) == hos.HOS_EINVAL
    assert f(FAKE, 0, ph, FAKE, FAKE, FAKE + 8, FAKE, wsb, None) == hos.HOS_EINVAL
    bad = plan.host.copy()
    bad[0] = 0   # not a plan
    assert f(FAKE, 0, bad.ctypes.data, FAKE, FAKE, FAKE, FAKE, wsb, None) == hos.HOS_EINVAL
    g = lib.hos_bispectrum_loss_fwd
    assert g(FAKE, 0, ph, FAKE, None, FAKE, FAKE, FAKE, wsb, None) == hos.HOS_EINVAL
    mixed = hos.BatchPlan([3000, 2000], [20, 21])
    assert g(FAKE, 0, mixed.host.ctypes.data, FAKE, FAKE, FAKE, FAKE, FAKE,
             mixed.info["ws_bytes"], None) == hos.HOS_EINVAL   # one target needs one M
    b = lib.hos_bispectrum_loss_bwd
    fwd_only = hos.BatchPlan([3000, 2000], [20, 20])
    assert b(FAKE, 0, fwd_only.host.ctypes.data, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
             fwd_only.info["ws_bytes"], None) == hos.HOS_EINVAL  # no adjoint buffers
    assert b(FAKE, 0, ph, FAKE, FAKE, FAKE, FAKE, FAKE + 2, FAKE, wsb, None) == hos.HOS_EINVAL


def test_tile_choice_moves_series_between_classes():
    n, M = [5000, 5000, 5000], [64, 64, 200]
    base = hos.BatchPlan(n, M, path="split_fp16")
    assert list(base.series()[:, 7]) == [0, 0, 1]
    forced = hos.BatchPlan(n, M, path="split_fp16", tile={64: 4, 200: 2})
    assert list(forced.series()[:, 7]) == [1, 1, 0]
    per = hos.BatchPlan(n, M, path="split_fp16", tile=[2, 4, 0])
    assert list(per.series()[:, 7]) == [0, 1, 1]
    with pytest.raises(hos.HosError):
        hos.BatchPlan(n, M, path="fp32", tile=[2, 2, 2])     # FP32 has 4 x 4 tiles only
    with pytest.raises(hos.HosError):
        hos.BatchPlan(n, M, path="split_fp16", tile=[3, 0, 0])
    # the split of a forced plan still covers every chunk once
    for cls in (0, 1):
        it = forced.items(cls)
        keys = set()
        for row in it:
            for ch in range(row[5], row[6]):
                key = (row[2], row[3], row[4], ch)
                assert key not in keys
                keys.add(key)


def test_tune_module_imports():
    from paper_1805_11775_amd import tune
    assert list(tune.DEFAULT_EDGES) == sorted(tune.DEFAULT_EDGES)
    assert tune.DEFAULT_EDGES[0] <= 1024 and tune.DEFAULT_EDGES[-1] > 65536


def test_segments_plan_and_validation():
    """HOS_PLAN_SEGMENTS needs one M; hos_bispectrum_segments checks its
    plan and outputs before touching a device."""
    with pytest.raises(hos.HosError):
        hos.BatchPlan([1000, 1000], [20, 21], segments=True)
    seg = hos.BatchPlan([1000] * 4, [20] * 4, segments=True)
    plain = hos.BatchPlan([1000] * 4, [20] * 4)
    assert seg.info["ws_bytes"] > plain.info["ws_bytes"]
    f = hos.lib().hos_bispectrum_segments
    wsb = seg.info["ws_bytes"]
    ph = seg.host.ctypes.data
    assert f(FAKE, 0, ph, FAKE, FAKE, FAKE, FAKE, wsb - 1, None) == hos.HOS_EWORKSPACE
    assert f(FAKE, 0, ph, FAKE, None, None, FAKE, wsb, None) == hos.HOS_EINVAL
    assert f(FAKE, 0, ph, FAKE, FAKE, FAKE + 8, FAKE, wsb, None) == hos.HOS_EINVAL
    assert f(FAKE, 0, plain.host.ctypes.data, FAKE, FAKE, FAKE, FAKE,
             plain.info["ws_bytes"], None) == hos.HOS_EINVAL     # plan without the flag
    assert f(None, 0, ph, FAKE, FAKE, FAKE, FAKE, wsb, None) == hos.HOS_EINVAL


def _tune_args(Ms, edges, series=8):
    Mc = (ctypes.c_int32 * len(Ms))(*Ms)
    Ec = (ctypes.c_int64 * len(edges))(*edges)
    return Mc, len(Ms), Ec, len(edges) - 1, series


@pytest.mark.parametrize("Ms,edges,series,code", [
    ([32, 128], [1024, 4096, 65537], 8, hos.HOS_OK),
    ([32], [1024, 1024], 8, hos.HOS_EINVAL),          # empty bucket
    ([32], [4096, 1024], 8, hos.HOS_EINVAL),          # decreasing edges
    ([2000], [1024, 65537], 8, hos.HOS_EINVAL),       # lag beyond the batch limit
    ([500], [100, 400], 8, hos.HOS_EINVAL),           # lag not below the lengths
    ([32], [1024, 4096], 0, hos.HOS_EINVAL),          # no series
])
def test_tune_validation_before_device(Ms, edges, series, code):
    """hos_tune's sizes are checked on the host; the workspace query covers
    the largest synthetic batch and plan."""
    Mc, nM, Ec, nb, se = _tune_args(Ms, edges, series)
    b = ctypes.c_size_t(0)
    assert hos.lib().hos_tune_workspace(1, Mc, nM, Ec, nb, se, ctypes.byref(b)) == code
    if code == hos.HOS_OK:
        assert b.value > 8 * (edges[-1] - 1) * 4
    tiles = (ctypes.c_int32 * 8)()
    ms = (ctypes.c_float * 16)()
    st = hos.lib().hos_tune(1, Mc, nM, Ec, nb, se, 3, ctypes.c_void_p(0x10000), 16, tiles, ms,
                            None)
    assert st == (hos.HOS_EWORKSPACE if code == hos.HOS_OK else code)


def test_tuned_table_lookup():
    """tiles_for maps each series to its lag's row and its length's bucket;
    the shipped table covers the batch workload's lags on every path."""
    from paper_1805_11775_amd import tune
    table = {"edges": [1024, 4096, 65537], "choices": {32: [2, 4], 256: [4, 2]}}
    assert tune.tiles_for([1024, 4095, 4096, 65536, 3000], [32, 32, 32, 256, 64], table) == \
        [2, 2, 4, 2, 0]
    for path in ("split_fp16", "split_bf16", "fp32"):
        t = tune.load("gfx950:256:" + path)
        assert t is not None and sorted(t["choices"]) == [32, 64, 128, 256]
        assert all(v in ((4,) if path == "fp32" else (2, 4))
                   for row in t["choices"].values() for v in row)


def test_batch_series_count_bound():
    """The series index is a grid dimension of the per-series kernels, so a
    plan takes at most 65535 series (refused on the host before any launch)."""
    import ctypes
    import numpy as np
    for count, want in ((65535, hos.HOS_OK), (65536, hos.HOS_EINVAL)):
        n = np.full(count, 64, dtype=np.int64)
        M = np.zeros(count, dtype=np.int32)
        pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        st = hos.lib().hos_batch_plan_size(
            count, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            M.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), hos.HOS_WIN_PARZEN,
            hos.HOS_PATH_SPLIT_FP16, 0, None, ctypes.byref(pb), ctypes.byref(wb))
        assert st == want, (count, st)
