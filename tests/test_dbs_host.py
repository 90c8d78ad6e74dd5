"""Host-side checks of the direct method's entry points: validation before
any HIP call, and the launch plan -- the strips and row runs of the
smoothing kernel cover every principal-domain point exactly once, which a
replay of the kernel's loop order (entering and leaving rows, window sums
as prefix differences) confirms against the oracle on small grids."""
import numpy as np
import pytest

import oracle
import paper_1805_11775_amd as hos
import synth

FAKE = 0x10000


@pytest.mark.parametrize("kw,code", [
    (dict(P=1), hos.HOS_EINVAL),
    (dict(P=7 * 16), hos.HOS_EINVAL),          # prime factor 7
    (dict(P=131072, n=1 << 18), hos.HOS_EINVAL),  # beyond the part-length limit
    (dict(n=100, P=128), hos.HOS_EINVAL),      # no whole part
    (dict(M3=0), hos.HOS_EINVAL),
    (dict(M3=129), hos.HOS_EINVAL),            # box wider than the grid
    (dict(M3=2049, P=4096), hos.HOS_EINVAL),   # beyond one strip
    (dict(flags=2), hos.HOS_EINVAL),
    (dict(dtype=3), hos.HOS_EINVAL),
    (dict(x=None), hos.HOS_EINVAL),
    (dict(B=FAKE + 8), hos.HOS_EINVAL),        # complex128 output not 16-byte aligned
    (dict(ws=FAKE + 64), hos.HOS_EINVAL),
    (dict(ws_bytes=100), hos.HOS_EWORKSPACE),
])
def test_validation_before_device(kw, code):
    a = dict(x=FAKE, dtype=hos.HOS_F32, n=4096, P=128, M3=9, flags=0, B=FAKE, ws=FAKE,
             ws_bytes=1 << 40)
    a.update(kw)
    st = hos.hos_dbs(a["x"], a["dtype"], a["n"], a["P"], a["M3"], a["flags"], a["B"],
                     a["ws"], a["ws_bytes"], None)
    assert st == code


@pytest.mark.parametrize("seg,strip", [(-1, 0), (0, 256), (0, 1000), (0, 512)])
def test_timed_rejects_bad_tuning(seg, strip):
    M3 = 600 if strip == 512 else 9           # a strip narrower than the box
    st, _ = hos.hos_dbs_timed(FAKE, 0, 4096, 2048, M3, 0, FAKE, FAKE, 1 << 40, None,
                              seg_rows=seg, strip_w=strip)
    assert st == hos.HOS_EINVAL


@pytest.mark.parametrize("n,P,M3", [(65536, 65536, 1023), (1 << 20, 1024, 33), (200, 16, 3),
                                    (12000, 6000, 100), (4096, 4096, 2048), (10, 2, 2)])
def test_plan(n, P, M3):
    info = hos.hos_dbs_plan_info(n, P, M3)
    assert info["K"] == n // P and info["mode"] == (0 if n // P == 1 else 1)
    assert info["P1"] * info["P2"] == P and max(info["P1"], info["P2"]) <= 4096
    H = (P - 1) // 2
    r = np.arange(H + 1)
    assert info["npd"] == np.sum(np.minimum(r, H - r) + 1)
    if P <= 6000:
        assert info["npd"] == len(oracle.pd_indices(P)[0])
    W, TW = info["W"], info["TW"]
    assert TW == W - M3 + 1 and TW >= 1
    assert info["NS"] * TW >= H // 2 + 1 > (info["NS"] - 1) * TW    # strips cover k2 <= H/2
    assert info["rows"] == sum(H - 2 * s * TW + 1 for s in range(info["NS"]))
    assert info["NWG"] * info["R"] >= info["rows"] > (info["NWG"] - 1) * info["R"]
    if info["mode"] == 1:
        assert info["G"] * info["Kg"] >= info["K"] > (info["G"] - 1) * info["Kg"]
        assert info["SR"] == H + M3 and info["SC"] >= (info["NS"] - 1) * TW + W
    assert info["ws_bytes"] == hos.hos_dbs_workspace(n, P, M3)


def _pd_row_off(r, H):
    m = H // 2
    tri = lambda t: t * (t + 1) // 2
    return tri(r) if r <= m + 1 else tri(m + 1) + tri(H - m) - tri(H + 1 - r)


def _replay(x, P, M3, seg_rows=0, strip_w=0):
    """The smoothing kernel's work split and loop order in numpy: the
    strips' rows end to end, cut into runs of R rows per workgroup."""
    info = hos.hos_dbs_plan_info(x.size, P, M3, seg_rows, strip_w)
    K, W, TW, R = info["K"], info["W"], info["TW"], info["R"]
    lo, H = M3 // 2, (P - 1) // 2
    hi = M3 - 1 - lo
    F = np.array([np.fft.fft(x[i * P:(i + 1) * P] - x[i * P:(i + 1) * P].mean())
                  for i in range(K)])
    out = np.full(info["npd"], np.nan, dtype=np.complex128)
    first = lambda s: s * (H + 1) - TW * s * (s - 1)

    def run(c0, ra, rb):
        T, qa = rb - ra + M3 - 1, ra - lo
        cw = c0 - lo + np.arange(W)

        def hsum(q):
            u = np.sum(F[:, q % P][:, None] * F[:, cw % P] * np.conj(F[:, (q + cw) % P]), 0)
            pf = np.concatenate([[0], np.cumsum(u)])
            return pf[np.arange(TW) + M3] - pf[np.arange(TW)]
        v = np.zeros(TW, dtype=np.complex128)
        for st in range(T):
            v = v + hsum(qa + st) - (hsum(qa + st - M3) if st >= M3 else 0)
            if st >= M3 - 1:
                r = qa + st - hi
                c = c0 + np.arange(TW)
                c = c[c <= min(r, H - r)]
                idx = _pd_row_off(r, H) + c
                assert np.isnan(out[idx]).all()
                out[idx] = v[:c.size] / (K * P * M3 * M3)

    for w in range(info["NWG"]):
        a, b = w * R, min(w * R + R, info["rows"])
        while a < b:
            s = max(k for k in range(info["NS"]) if first(k) <= a)
            c0 = s * TW
            ra = c0 + a - first(s)
            rb = min(c0 + b - first(s), H - c0 + 1)
            run(c0, ra, rb)
            a += rb - ra
    return out


@pytest.mark.parametrize("n,P,M3,seg,strip", [
    (64, 64, 5, 0, 0), (300, 30, 4, 0, 0), (97, 32, 1, 0, 0), (40, 40, 40, 0, 0),
    (700, 300, 7, 0, 0), (700, 300, 7, 5, 0), (1200, 600, 257, 0, 0), (3000, 3000, 300, 64, 512),
    (2000, 2000, 5, 0, 1024)])
def test_kernel_loop_order_replay(n, P, M3, seg, strip):
    x = synth.iid_exp_centered(n, 3)
    got = _replay(x, P, M3, seg, strip)
    assert not np.isnan(got).any()
    if P <= 300:
        ref = oracle.dbs(x, P, M3)
    else:
        k1, k2 = oracle.pd_indices(P)
        pick = np.arange(0, k1.size, 97)
        ref, got = oracle.dbs_at(x, P, M3, k1[pick], k2[pick]), got[pick]
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
