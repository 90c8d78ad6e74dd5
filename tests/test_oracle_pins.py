"""Pins of the FP64 oracle to facts outside itself.

Each test checks the oracle against something the mathematics or the paper
fixes -- a closed form, an exact identity with a textbook FFT, a symmetry the
brute-force code does not use, a hand-worked value, or a population cumulant
of a process with a known answer -- chosen so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails one of them.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_gold(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.asarray(rows)


# ---------------------------------------------------------------- c3 ----
def test_c3_matches_literal_loops_tiny():
    """C core vs an independently spelled pure-Python loop (n = 23, M = 6)."""
    x = synth.iid_exp_centered(23, 11)
    xt = brute.center(list(x))
    c = oracle.c3_square(x, 6)
    for w1 in range(-6, 7):
        for w2 in range(-6, 7):
            assert abs(c[w1 + 6, w2 + 6] - brute.c3(xt, w1, w2)) < 1e-14


def test_c3_constant_uncentered_closed_form():
    """x_t = a: c3(w) = a^3 (n - span(w)) / n, all lags of the square."""
    n, M, a = 37, 9, 1.75
    c = oracle.c3_square(np.full(n, a), M, centered=False)
    expect = a ** 3 * (n - oracle.span3(M)) / n
    np.testing.assert_allclose(c, expect, rtol=0, atol=1e-13)


def test_c3_constant_centered_is_zero():
    c = oracle.c3_square(np.full(50, 3.25), 7)
    assert np.max(np.abs(c)) == 0.0


def test_c3_impulse_uncentered():
    """x = A delta_{t0}: c3 = A^3/n at the origin only; B is flat."""
    n, M, A, t0 = 40, 8, 2.0, 17
    x = np.zeros(n)
    x[t0] = A
    c = oracle.c3_square(x, M, centered=False)
    expect = np.zeros_like(c)
    expect[M, M] = A ** 3 / n
    np.testing.assert_allclose(c, expect, atol=1e-15)
    _, B = oracle.bispectrum(x, M, 2 * M, "parzen", centered=False)
    np.testing.assert_allclose(B, np.full_like(B, A ** 3 / n), atol=1e-14)


def _impulse_centered_closed_form(n, A, t0, w1, w2):
    """x~_t = q + p delta_{t,t0} with p = A, q = -A/n.  Expand the product of
    the three factors over the subsets S of factor positions taking p:
    S empty contributes q^3 |I(w)|; otherwise every offset in S must be equal
    and t = t0 - offset must lie in the valid range I(w)."""
    offs = (0, w1, w2)
    lo = -min(offs)
    hi = n - 1 - max(offs)
    count = max(0, hi - lo + 1)
    p, q = A, -A / n
    total = 0.0
    for r in range(4):
        for S in itertools.combinations(range(3), r):
            coef = p ** len(S) * q ** (3 - len(S))
            if not S:
                total += coef * count
                continue
            o = {offs[k] for k in S}
            if len(o) != 1:
                continue
            t = t0 - o.pop()
            if lo <= t <= hi:
                total += coef
    return total / n


def test_c3_impulse_centered_closed_form():
    n, M, A, t0 = 29, 7, 1.5, 10
    x = np.zeros(n)
    x[t0] = A
    c = oracle.c3_square(x, M)
    for w1 in range(-M, M + 1):
        for w2 in range(-M, M + 1):
            e = _impulse_centered_closed_form(n, A, t0, w1, w2)
            assert abs(c[w1 + M, w2 + M] - e) < 1e-14, (w1, w2)


def test_c3_six_fold_symmetry():
    """c3(w1,w2) = c3(w2,w1) = c3(-w1,w2-w1) = c3(w1-w2,-w2) = c3(-w2,w1-w2)
    = c3(w2-w1,-w1), checked where every image stays inside the square."""
    M = 10
    x = synth.quadratic_process(300, 5)
    c = oracle.c3_square(x, M)
    f = lambda a, b: c[a + M, b + M]
    for w1 in range(-M, M + 1):
        for w2 in range(-M, M + 1):
            imgs = [(w2, w1), (-w1, w2 - w1), (w1 - w2, -w2), (-w2, w1 - w2),
                    (w2 - w1, -w1)]
            for a, b in imgs:
                if abs(a) <= M and abs(b) <= M:
                    assert abs(f(a, b) - f(w1, w2)) < 1e-15


def test_c3_all_lag_sum_is_cube_of_sum():
    """sum over all lags |w| <= n-1 of n c3(w) = (sum_t x_t)^3."""
    x = synth.iid_gauss(12, 3) + 0.3
    n = x.size
    c = oracle.c3_square(x, n - 1, centered=False)
    assert abs(c.sum() * n - x.sum() ** 3) < 1e-11
    cc = oracle.c3_square(x, n - 1)  # centred: the cube of 0
    assert abs(cc.sum()) < 1e-12


@pytest.mark.parametrize("N", [19, 24, 7])
def test_direct_equals_indirect_bispectrum(N):
    """No window and M = n-1: the lag-domain DFT equals (1/n) X(k1) X(k2)
    X*(k1+k2) with X the N-point FFT of the centred record -- the raw
    bispectrum of Algorithm DBS with one part and the conjugate on the third
    factor.  N = 7 checks
    the folding of aliased lags."""
    x = synth.iid_exp_centered(10, 21)
    n = x.size
    _, B = oracle.bispectrum(x, n - 1, N, window="none")
    xt = x - x.mean()
    if N >= n:
        X = np.fft.fft(xt, N)
    else:  # fold the record onto the N-grid before the FFT
        X = np.fft.fft(np.bincount(np.arange(n) % N, weights=xt, minlength=N))
    k = np.arange(N)
    ref = X[:, None] * X[None, :] * np.conj(X[(k[:, None] + k[None, :]) % N]) / n
    np.testing.assert_allclose(B, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_bispectrum_symmetries():
    """B(k1,k2) = B(k2,k1) = conj B(-k1,-k2) = B(k1, -k1-k2) (mod N)."""
    M, N = 12, 24
    x = synth.quadratic_process(400, 8)
    _, B = oracle.bispectrum(x, M, N)
    k = np.arange(N)
    K1, K2 = np.meshgrid(k, k, indexing="ij")
    tol = 1e-13 * np.abs(B).max()
    np.testing.assert_allclose(B, B.T, atol=tol)
    np.testing.assert_allclose(B, np.conj(B[(-K1) % N, (-K2) % N]), atol=tol)
    np.testing.assert_allclose(B, B[K1, (-K1 - K2) % N], atol=tol)


# ---------------------------------------------------------- window ----
def test_parzen_hand_values():
    g = _load_gold("parzen_points.txt")
    for m, L, d in g:
        assert oracle.parzen(m, int(L)) == pytest.approx(d, abs=1e-15)


def test_parzen_zero_scale_limit():
    """M = 0 leaves the single lag 0: the window must keep it (weight 1)."""
    assert oracle.parzen(0, 0) == 1.0 and oracle.parzen(3, 0) == 0.0
    assert oracle.window3(0)[0, 0] == 1.0


def test_window3_symmetry_and_support():
    M = 16
    W = oracle.window3(M)
    c = W[M, M]
    assert c == 1.0
    f = lambda a, b: W[a + M, b + M]
    for w1 in range(-M, M + 1):
        for w2 in range(-M, M + 1):
            if abs(w1 - w2) <= M:
                assert abs(f(w2, w1) - f(w1, w2)) < 1e-15
                assert abs(f(-w1, w2 - w1) - f(w1, w2)) < 1e-15
            else:
                assert f(w1, w2) == 0.0


# ---------------------------------------------------- c2 / c4 -----
def test_c4_matches_literal_loops_tiny():
    x = synth.iid_exp_centered(17, 4)
    xt = brute.center(list(x))
    M = 3
    c = oracle.c4_cube(x, M)
    for t in itertools.product(range(-M, M + 1), repeat=3):
        i = tuple(v + M for v in t)
        assert abs(c[i] - brute.c4(xt, *t)) < 1e-13


def test_c2_direct_equals_indirect():
    """sum_d c2(d) e^{-i w k d} over |d| <= n-1 equals |X(k)|^2 / n."""
    x = synth.iid_gauss(13, 6)
    n = x.size
    c = oracle.c2(x, n - 1)
    N = 32
    d = np.arange(-(n - 1), n)
    full = np.concatenate([c[:0:-1], c])
    k = np.arange(N)[:, None]
    S = (full[None, :] * np.exp(-2j * np.pi * k * d[None, :] / N)).sum(1)
    X = np.fft.fft(x - x.mean(), N)
    np.testing.assert_allclose(S, np.abs(X) ** 2 / n, atol=1e-12)


def test_m4_direct_equals_indirect():
    """3D DFT of m4 over all lags equals (1/n) X(k1)X(k2)X(k3)X*(k1+k2+k3)."""
    x = synth.iid_exp_centered(7, 9)
    n = x.size
    M = n - 1
    t = np.arange(-M, M + 1)
    T1, T2, T3 = np.meshgrid(t, t, t, indexing="ij")
    m4 = oracle.m4_at(x, T1, T2, T3).reshape(T1.shape)
    N = 13
    F = np.fft.fftn(oracle.place_circular(m4, M, N))
    X = np.fft.fft(x - x.mean(), N)
    k = np.arange(N)
    K1, K2, K3 = np.meshgrid(k, k, k, indexing="ij")
    ref = X[K1] * X[K2] * X[K3] * np.conj(X[(K1 + K2 + K3) % N]) / n
    np.testing.assert_allclose(F, ref, atol=1e-12 * np.abs(ref).max())


def _pairings(pts):
    """Number of ways the 4 points split into two pairs of equal times,
    counting only the three pairings the c2 corrections use."""
    p0, p1, p2, p3 = pts
    return int(p0 == p1 and p2 == p3) + int(p0 == p2 and p1 == p3) + \
        int(p0 == p3 and p1 == p2)


def test_c4_impulse_uncentered_closed_form():
    """x = A delta_{t0}: m4 = A^4/n at the origin, c2(d) = A^2/n at d = 0, so
    c4(t) = A^4/n [t = 0] - A^4/n^2 (number of equal-time pairings)."""
    n, M, A, t0 = 20, 4, 1.3, 9
    x = np.zeros(n)
    x[t0] = A
    c = oracle.c4_cube(x, M, centered=False)
    for t in itertools.product(range(-M, M + 1), repeat=3):
        e = -A ** 4 / n ** 2 * _pairings((0,) + t)
        if t == (0, 0, 0):
            e += A ** 4 / n
        assert abs(c[tuple(v + M for v in t)] - e) < 1e-15, t


def test_c4_24_fold_symmetry():
    M = 4
    x = synth.cubic_process(120, 2)
    c = oracle.c4_cube(x, M)
    f = lambda t: c[t[0] + M, t[1] + M, t[2] + M]
    for t in itertools.product(range(-M, M + 1), repeat=3):
        pts = (0,) + t
        for origin in pts:
            rest = list(pts)
            rest.remove(origin)
            for perm in itertools.permutations(rest):
                img = tuple(p - origin for p in perm)
                if max(abs(v) for v in img) <= M:
                    assert abs(f(img) - f(t)) < 1e-15


# -------------------------------------------- population cumulants --
def _batch_se(prod, nb=64):
    """Standard error of the mean of a weakly dependent series (batch means)."""
    m = prod[: prod.size // nb * nb].reshape(nb, -1).mean(1)
    return m.std(ddof=1) / np.sqrt(nb)


def test_exp_third_and_fourth_cumulant():
    """Centred Exp(1): kappa3 = 2, kappa4 = 6; zero off the origin."""
    n = 1 << 18
    x = synth.iid_exp_centered(n, 77)
    xt = oracle.center(x)
    c3 = oracle.c3_at(x, [0, 1, 2, 0], [0, 1, 0, 3])
    se = _batch_se(xt ** 3)
    assert abs(c3[0] - 2.0) < 6 * se
    for v in c3[1:]:
        assert abs(v) < 6 * se
    c4 = oracle.c4_at(x, [0, 1], [0, 2], [0, 3])
    se4 = _batch_se(xt ** 4)
    assert abs(c4[0] - 6.0) < 6 * se4
    assert abs(c4[1]) < 6 * se4


def test_gaussian_cumulants_vanish():
    """Gaussian input: c3 = c4 = 0 (Section 1, the Gaussianity test); the
    fourth moment at the origin (about 3) must cancel against the c2 terms."""
    n = 1 << 18
    x = synth.iid_gauss(n, 99)
    xt = oracle.center(x)
    c3 = oracle.c3_at(x, [0, 1, 3], [0, 2, -1])
    se = _batch_se(xt ** 3)
    assert np.all(np.abs(c3) < 6 * se)
    c4 = oracle.c4_at(x, [0, 1, 0], [0, 1, 2], [0, 1, 0])
    se4 = _batch_se(xt ** 4)
    assert np.all(np.abs(c4) < 6 * se4)


def test_quadratic_process_c3():
    g = _load_gold("quadratic_process_c3.txt")
    n = 1 << 18
    x = synth.quadratic_process(n, 1234)
    xt = oracle.center(x)
    c = oracle.c3_at(x, g[:, 0], g[:, 1])
    for (w1, w2, true), v in zip(g, c):
        w1, w2 = int(w1), int(w2)
        lo = max(0, -w1, -w2)
        hi = n - max(0, w1, w2)
        se = _batch_se(xt[lo:hi] * xt[lo + w1:hi + w1] * xt[lo + w2:hi + w2])
        assert abs(v - true) < 6 * se + 1e-12, (w1, w2, v, true, se)


def test_cubic_process_c4():
    g = _load_gold("cubic_process_c4.txt")
    n = 1 << 18
    x = synth.cubic_process(n, 4321)
    xt = oracle.center(x)
    c = oracle.c4_at(x, g[:, 0], g[:, 1], g[:, 2])
    for (t1, t2, t3, true), v in zip(g, c):
        t = (int(t1), int(t2), int(t3))
        lo = max(0, -min(t))
        hi = n - max(0, max(t))
        prod = xt[lo:hi].copy()
        for s in t:
            prod = prod * xt[lo + s:hi + s]
        se = _batch_se(prod)
        assert abs(v - true) < 7 * se + 1e-12, (t, v, true, se)


# ------------------------------------------------ principal domain --
def test_principal_domain_count_and_shape():
    """0 <= k2 <= k1, k1 + k2 < N/2: with h = N/2 even there are
    h^2/4 + h/2 points (16,512 at N = 512)."""
    for N in (8, 12, 128, 512):
        k1, k2 = oracle.pd_indices(N)
        h = N // 2
        if h % 2 == 0:
            assert k1.size == h * h // 4 + h // 2
        assert np.all(k2 <= k1) and np.all(k1 + k2 < N / 2) and np.all(k2 >= 0)
    assert oracle.pd_indices(512)[0].size == 16512


# --------------------------------------------------------------------------
# Bispectrum-matching loss and its gradient
# --------------------------------------------------------------------------
def _loss_case(n, M, N, seed, window="parzen"):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 0.3 * rng.standard_normal(n) ** 2
    npd = len(oracle.pd_indices(N)[0])
    target = 0.05 * (rng.standard_normal(npd) + 1j * rng.standard_normal(npd))
    return x, target


@pytest.mark.parametrize("n,M,N,window", [(48, 6, 12, "parzen"), (40, 6, 13, "none"),
                                          (33, 4, 9, "none")])
def test_loss_gradient_matches_central_differences(n, M, N, window):
    """L is a polynomial of degree 6 in x, so central differences with a small
    step agree with the exact gradient to O(h^2)."""
    x, target = _loss_case(n, M, N, 31 + n, window)
    g = oracle.bispectrum_loss_grad(x, M, N, target, window)
    h = 1e-5
    fd = np.empty(n)
    for j in range(n):
        xp = x.copy()
        xm = x.copy()
        xp[j] += h
        xm[j] -= h
        fd[j] = (oracle.bispectrum_loss(xp, M, N, target, window) -
                 oracle.bispectrum_loss(xm, M, N, target, window)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(g))


def test_loss_gradient_euler_identity():
    """With a zero target L(lambda x) = lambda^6 L(x) (c3 is cubic in the
    mean-removed series, which is linear in x), so <x, grad L> = 6 L."""
    x, _ = _loss_case(200, 10, 20, 5)
    target = np.zeros(len(oracle.pd_indices(20)[0]), dtype=np.complex128)
    L = oracle.bispectrum_loss(x, 10, 20, target)
    g = oracle.bispectrum_loss_grad(x, 10, 20, target)
    assert abs(np.dot(x, g) - 6.0 * L) < 1e-10 * 6.0 * L


def test_loss_gradient_shift_invariance():
    """Mean removal makes L(x + c) = L(x), so the gradient sums to zero; and
    the gradient of a batch is the per-series gradients stacked."""
    x, target = _loss_case(150, 12, 24, 6)
    y, _ = _loss_case(150, 12, 24, 7)
    g = oracle.bispectrum_loss_grad(np.stack([x, y]), 12, 24, target)
    assert abs(np.sum(g[0])) < 1e-12 * np.max(np.abs(g[0])) * x.size
    assert np.array_equal(g[1], oracle.bispectrum_loss_grad(y, 12, 24, target))
    assert abs(oracle.bispectrum_loss(np.stack([x, y]), 12, 24, target) -
               oracle.bispectrum_loss(x, 12, 24, target) -
               oracle.bispectrum_loss(y, 12, 24, target)) < 1e-12


def test_loss_gradient_at_indices_agrees_with_full():
    """The sampled form returns the full gradient's entries before the mean
    term: differences between indices agree exactly."""
    x, target = _loss_case(120, 8, 16, 9)
    g = oracle.bispectrum_loss_grad(x, 8, 16, target)
    idx = np.array([0, 5, 60, 119])
    ga = oracle.loss_grad_at(x, 8, 16, target, idx)
    assert np.allclose(ga - ga[0], g[idx] - g[idx[0]], rtol=0, atol=1e-13 * np.max(np.abs(g)))


def test_separable_window_hand_values():
    """Separable Parzen (the product over the lags only) against hand values:
    at L = 4, d(2) = 1 - 6/4 + 6/8 = 1/4 and d(4) = 0, so at (w1, w2) = (2, -2)
    the separable window is 1/16 while the full one (times d(w1 - w2) = d(4))
    is 0; at (1, 1) both are d(1)^2 (times d(0) = 1)."""
    M = 4
    ws, wf = oracle.window3(M, "separable"), oracle.window3(M, "parzen")
    d1 = 1 - 6 * (1 / 4) ** 2 + 6 * (1 / 4) ** 3
    assert ws[2 + M, -2 + M] == 0.0625 and wf[2 + M, -2 + M] == 0.0
    assert abs(ws[1 + M, 1 + M] - d1 * d1) < 1e-15 and abs(wf[1 + M, 1 + M] - d1 * d1) < 1e-15
    w4 = oracle.window4(M, "separable")
    assert abs(w4[2 + M, -2 + M, 1 + M] - 0.0625 * d1) < 1e-15
    assert oracle.window4(M, "parzen")[2 + M, -2 + M, 1 + M] == 0.0


def test_window4_hand_values():
    """W4 = product of d over the six pairwise differences of {0,t1,t2,t3}
    against hand-worked products at M = 8 (tests/golden/window4_points.txt):
    two lags whose six differences are non-zero and distinct, and six lags
    that vanish through exactly one factor each."""
    M = 8
    W = oracle.window4(M)
    for row in _load_gold("window4_points.txt"):
        t = tuple(int(v) for v in row[:3])
        t1, t2, t3 = t
        diffs = (abs(t1), abs(t2), abs(t3), abs(t2 - t1), abs(t3 - t1), abs(t3 - t2))
        assert diffs == tuple(int(v) for v in row[3:9]), t   # the fixture's own bookkeeping
        expect = row[9] / row[10]
        got = W[t1 + M, t2 + M, t3 + M]
        assert got == expect, (t, got, expect)


def test_window4_24_fold_symmetry_and_support():
    """W4 takes one value on each orbit of the 24-fold lag symmetry (any of
    the four offsets as origin, the other three in any order), and is zero
    exactly where the span of {0,t1,t2,t3} reaches M."""
    M = 6
    W = oracle.window4(M)
    f = lambda t: W[t[0] + M, t[1] + M, t[2] + M]
    for t in itertools.product(range(-M, M + 1), repeat=3):
        pts = (0,) + t
        span = max(pts) - min(pts)
        assert (f(t) == 0.0) == (span >= M), t
        for origin in pts:
            rest = list(pts)
            rest.remove(origin)
            for perm in itertools.permutations(rest):
                img = tuple(p - origin for p in perm)
                if max(abs(v) for v in img) <= M:
                    assert abs(f(img) - f(t)) < 1e-15, (t, img)


def test_c4_support_boundary():
    """c4_support keeps every lag of span M (equal to the literal loops there,
    and non-zero) and zeroes every lag of span M + 1 or more."""
    M = 3
    x = synth.cubic_process(40, 12)
    xt = brute.center(list(x))
    c = oracle.c4_support(x, M)
    kept = 0
    for t in itertools.product(range(-M, M + 1), repeat=3):
        pts = (0,) + t
        span = max(pts) - min(pts)
        v = c[tuple(v + M for v in t)]
        if span <= M:
            ref = brute.c4(xt, *t)
            assert abs(v - ref) < 1e-13, t
            if span == M:
                assert ref != 0.0
                kept += 1
        else:
            assert v == 0.0, t
    assert kept > 0


def test_trispectrum_hermitian_and_permutation_symmetry():
    """T from the oracle's own composition (c4 on its support, W4, 3-D DFT):
    T(k) = conj T(-k), T is invariant under permutations of (k1, k2, k3) and
    under k1 -> -k1-k2-k3 (the fourth frequency of the 24-fold symmetry)."""
    M, N = 5, 10
    x = synth.cubic_process(300, 13)
    _, T = oracle.trispectrum(x, M, N)
    k = np.arange(N)
    K1, K2, K3 = np.meshgrid(k, k, k, indexing="ij")
    tol = 1e-13 * np.abs(T).max()
    np.testing.assert_allclose(T, np.conj(T[(-K1) % N, (-K2) % N, (-K3) % N]), atol=tol)
    for perm in itertools.permutations(range(3)):
        np.testing.assert_allclose(T, T.transpose(perm), atol=tol)
    np.testing.assert_allclose(T, T[(-K1 - K2 - K3) % N, K2, K3], atol=tol)


def test_trispectrum_matches_direct_lag_sum():
    """At sampled frequencies T equals the direct sum over every lag of the
    cube of W4 c4 e^{-2 pi i <k, t>/N}, with W4 and c4 formed here from the
    literal loops and hand-expanded Parzen products (aliases included, N < 2M+1)."""
    M, N = 3, 5
    x = synth.cubic_process(60, 14)
    xt = brute.center(list(x))
    _, T = oracle.trispectrum(x, M, N)

    def d(m):
        r = abs(m) / M
        return 1 - 6 * r * r + 6 * r ** 3 if r <= 0.5 else (2 * (1 - r) ** 3 if r <= 1 else 0.0)

    lags = list(itertools.product(range(-M, M + 1), repeat=3))
    vals = []
    for t in lags:
        t1, t2, t3 = t
        w = d(t1) * d(t2) * d(t3) * d(t2 - t1) * d(t3 - t1) * d(t3 - t2)
        vals.append(w * brute.c4(xt, *t) if w != 0.0 else 0.0)
    for kk in [(0, 0, 0), (1, 2, 3), (4, 0, 2), (3, 3, 1)]:
        s = sum(v * np.exp(-2j * np.pi * (kk[0] * t[0] + kk[1] * t[1] + kk[2] * t[2]) / N)
                for v, t in zip(vals, lags))
        assert abs(s - T[kk]) < 1e-12 * np.abs(T).max(), kk


def test_bispectrum_full_square_region():
    """c3 is returned on the hexagon (corners 0) or, with full_square, at
    every lag of the square, the corners equal to the literal loops.  B
    transforms the windowed sample cumulant over the whole square whatever
    c3's region (Section 1, Problem Statement: the cumulant at every lag up
    to the maximum lag): at no window B minus the DFT of the hexagon part is
    the DFT of the corners, checked at one frequency against the corner
    lags summed one by one; the Parzen product vanishes on the corners."""
    n, M, N = 30, 5, 11
    x = synth.quadratic_process(n, 15)
    xt = brute.center(list(x))
    c_sq, B_sq = oracle.bispectrum(x, M, N, window="none", full_square=True)
    c_hx, B_hx = oracle.bispectrum(x, M, N, window="none")
    assert np.array_equal(B_sq, B_hx)
    B_hex_only = np.fft.fft2(oracle.place_circular(c_hx, M, N))
    corner = 0j
    k1, k2 = 2, 7
    for w1 in range(-M, M + 1):
        for w2 in range(-M, M + 1):
            v = brute.c3(xt, w1, w2)
            assert abs(c_sq[w1 + M, w2 + M] - v) < 1e-14
            if abs(w1 - w2) > M:
                assert c_hx[w1 + M, w2 + M] == 0.0
                assert v != 0.0
                corner += v * np.exp(-2j * np.pi * (k1 * w1 + k2 * w2) / N)
    assert abs((B_sq - B_hex_only)[k1, k2] - corner) < 1e-13
    # the separable window is nonzero on the corners too: d(w1) d(w2)
    _, B_sep = oracle.bispectrum(x, M, 2 * M, window="separable")
    W = oracle.window3(M, "separable")
    assert np.max(W[oracle.span3(M) > M]) > 0.0
    ref = np.fft.fft2(oracle.place_circular(c_sq * W, M, 2 * M))
    assert np.max(np.abs(B_sep - ref)) < 1e-15 * np.max(np.abs(ref))
    # the Parzen product vanishes on the corners: both regions give one B
    _, B1 = oracle.bispectrum(x, M, 2 * M, full_square=True)
    _, B2 = oracle.bispectrum(x, M, 2 * M)
    assert np.max(np.abs(B1 - B2)) < 1e-15 * np.max(np.abs(B2))
    Wp = oracle.window3(M, "parzen")
    assert np.all(Wp[oracle.span3(M) > M] == 0.0)


def test_trispectrum_uses_the_whole_cube_off_parzen():
    """T transforms the windowed c4 over the whole cube: with the separable
    window (nonzero where the span exceeds M) it differs from the transform
    of the span <= M part by the transform of the rest, checked at one
    frequency against those lags summed one by one from the literal loops."""
    n, M, N = 14, 3, 7
    x = synth.cubic_process(n, 16)
    xt = brute.center(list(x))
    c, T = oracle.trispectrum(x, M, N, window="separable")
    W = oracle.window4(M, "separable")
    T_support = np.fft.fftn(oracle.place_circular(c * W, M, N))
    kk = (1, 3, 2)
    rest = 0j
    lags = range(-M, M + 1)
    for t1 in lags:
        for t2 in lags:
            for t3 in lags:
                span = max(0, t1, t2, t3) - min(0, t1, t2, t3)
                if span > M:
                    w = W[t1 + M, t2 + M, t3 + M]
                    rest += w * brute.c4(xt, t1, t2, t3) * np.exp(
                        -2j * np.pi * (kk[0] * t1 + kk[1] * t2 + kk[2] * t3) / N)
                else:
                    assert abs(c[t1 + M, t2 + M, t3 + M] - brute.c4(xt, t1, t2, t3)) < 1e-14
    assert abs(rest) > 1e-6
    assert abs((T - T_support)[kk] - rest) < 1e-12 * np.max(np.abs(T))


# --------------------------------------------------------------------------
# The direct method (Algorithm DBS)
# --------------------------------------------------------------------------
def test_dbs_raw_is_dft_of_circular_triple_correlation():
    """F(k1)F(k2)conj(F(k1+k2))/P equals the unnormalised 2-D DFT of the
    circular third moment, computed here by brute force: pins the conjugate
    placement and the 1/P."""
    x = synth.iid_exp_centered(24, 3)
    raw = oracle.dbs_raw(x)
    c = oracle.c3_circular(x)
    P = x.size
    w = np.arange(P)
    E = np.exp(-2j * np.pi * np.outer(w, w) / P)
    assert np.max(np.abs(raw - E @ c @ E.T)) < 1e-12 * np.max(np.abs(raw))


def test_dbs_smoothing_box():
    """A unit impulse at (p1, p2) spreads 1/M3^2 over exactly the points whose
    window contains it: k - n = p for n in [-floor(M3/2), M3-1-floor(M3/2)],
    with wrap-around; a constant grid is unchanged."""
    P = 16
    for M3 in (1, 4, 5):
        C = np.zeros((P, P), dtype=np.complex128)
        C[3, 14] = 1.0
        S = oracle.dbs_smooth(C, M3)
        lo = M3 // 2
        expect = np.zeros((P, P))
        for n1 in range(-lo, M3 - lo):
            for n2 in range(-lo, M3 - lo):
                expect[(3 - n1) % P, (14 - n2) % P] = 1.0 / M3 ** 2
        assert np.allclose(S, expect, atol=1e-15)
        assert np.allclose(oracle.dbs_smooth(np.full((P, P), 2.5 + 1j), M3), 2.5 + 1j)


def test_dbs_averaging_and_mean_removal():
    """K copies of one part give that part's result; adding a constant to a
    part changes nothing; trailing samples beyond K P are ignored."""
    part = synth.quadratic_process(32, 4)
    one = oracle.dbs(part, 32, 3)
    x = np.concatenate([part, part + 7.0, part - 1.5, [9.0] * 5])
    assert np.allclose(oracle.dbs(x, 32, 3), one, rtol=0, atol=1e-12 * np.max(np.abs(one)))


def test_dbs_matches_indirect_with_one_part_and_no_smoothing():
    """K = 1, M3 = 1, with the part zero-padded to length >= 2n-1 outside the
    estimator: the direct raw bispectrum of the padded part is n/N' times the
    indirect B of the unpadded series with no window and M = n-1 (the
    circular and the zero-padded third moments then coincide)."""
    x = synth.iid_exp_centered(20, 8)
    n, N = x.size, 40
    xt = x - np.mean(x)
    padded = np.concatenate([xt, np.zeros(N - n)])
    raw = oracle.dbs_raw(padded)      # its mean removal shifts nothing: mean(padded) = 0
    _, B = oracle.bispectrum(x, n - 1, N, window="none")
    assert np.max(np.abs(raw * N / n - B)) < 1e-10 * np.max(np.abs(B))


def test_dbs_at_matches_dbs():
    """The sampled form agrees with the whole-grid form, K = 3, odd and even
    box sizes, including points whose box wraps around the grid."""
    x = synth.iid_exp_centered(3 * 30 + 7, 12)
    k1, k2 = oracle.pd_indices(30)
    for M3 in (1, 4, 7):
        full = oracle.dbs(x, 30, M3)
        pick = np.arange(0, k1.size, 5)
        got = oracle.dbs_at(x, 30, M3, k1[pick], k2[pick])
        assert np.max(np.abs(got - full[pick])) < 1e-12 * np.max(np.abs(full))


# --------------------------------------------------------------------------
# Segment averaging for the indirect estimator
# --------------------------------------------------------------------------
def test_segments_lag_zero_is_mean_central_third_moment():
    """M = 0: c3(0,0) is the average over segments of each segment's third
    central moment (scipy's, with 1/P)."""
    from scipy import stats
    x = synth.iid_exp_centered(5 * 40 + 3, 21)
    c, _ = oracle.bispectrum_segments(x, 40, 0, 2, window="none")
    expect = np.mean([stats.moment(x[i * 40:(i + 1) * 40], 3) for i in range(5)])
    assert abs(c[0, 0] - expect) < 1e-13 * abs(expect)


def test_segments_centre_each_segment():
    """A different constant added to each segment changes nothing; K copies
    of one segment give that segment's estimate; trailing samples are
    ignored."""
    seg = synth.quadratic_process(50, 9)
    x = np.concatenate([seg + 3.0, seg - 7.5, seg, [100.0] * 7])
    c, B = oracle.bispectrum_segments(x, 50, 6, 12)
    c1, B1 = oracle.bispectrum(seg, 6, 12)
    assert np.max(np.abs(c - c1)) < 1e-12 * np.max(np.abs(c1))
    assert np.max(np.abs(B - B1)) < 1e-12 * np.max(np.abs(B1))


def test_segments_match_direct_method_parts():
    """No window, M = P - 1, N = 2P: each segment's indirect B equals N/P
    times the direct method's raw product of the segment centred and
    zero-padded to N, so the segment average on the principal domain is N/P
    times the direct method over those padded parts with no smoothing."""
    P, K, N = 12, 4, 24
    x = synth.iid_exp_centered(P * K, 31)
    _, B = oracle.bispectrum_segments(x, P, P - 1, N, window="none")
    parts = []
    for i in range(K):
        s = x[i * P:(i + 1) * P]
        parts.append(np.concatenate([s - s.mean(), np.zeros(N - P)]))
    direct = oracle.dbs(np.concatenate(parts), N, 1)
    k1, k2 = oracle.pd_indices(N)
    assert np.max(np.abs(B[k1, k2] - direct * N / P)) < 1e-10 * np.max(np.abs(direct))


# --------------------------------------------------------------------------
# Order five
# --------------------------------------------------------------------------
def test_c5_matches_literal_loops():
    """The C core against the pure-Python literal loops on a tiny record,
    every lag of the hypercube M = 2 plus lags reaching past the record."""
    x = synth.iid_exp_centered(9, 17)
    c = oracle.c5_hyper(x, 2)
    xt = brute.center(list(x))
    rng = np.random.default_rng(0)
    for t in [tuple(v) for v in rng.integers(-2, 3, (60, 4))] + [(0, 0, 0, 0), (2, -2, 1, 0)]:
        assert abs(c[tuple(np.asarray(t) + 2)] - brute.c5(xt, *t)) < 1e-13
    for t in [(8, 0, 0, 0), (-8, 3, 1, 0), (5, -4, 0, 2)]:
        assert abs(oracle.c5_at(x, *[[v] for v in t])[0] - brute.c5(xt, *t)) < 1e-13


def test_c5_lag_zero_is_fifth_cumulant_of_the_sample():
    """At the origin c5 is the fifth cumulant of the sample's own
    distribution, mu5 - 10 mu2 mu3 for central moments (scipy's)."""
    from scipy import stats
    x = synth.quadratic_process(300, 2)
    mu = [stats.moment(x, k) for k in (2, 3, 5)]
    got = oracle.c5_at(x, [0], [0], [0], [0])[0]
    assert abs(got - (mu[2] - 10 * mu[0] * mu[1])) < 1e-12 * abs(mu[2])


def test_c5_uncentred_impulse_closed_form():
    """x = A delta_{t0}, no mean removal: m5 = A^5/n at the origin only,
    c2 = A^2/n at lag 0, c3 = A^3/n at (0,0); so c5 = A^5/n [all offsets
    equal] - (A^2/n)(A^3/n) times the number of pair / triple splits of the
    five offsets whose pair and triple are each constant."""
    n, A, M = 40, 1.7, 2
    x = np.zeros(n)
    x[20] = A
    c = oracle.c5_hyper(x, M, centered=False)
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
    assert np.max(np.abs(c - expect)) < 1e-14


def test_c5_symmetries_and_zero_for_constants():
    """The 120-fold symmetry (permutations of t1..t4 and the shift
    (t1..t4) -> (-t1, t2-t1, t3-t1, t4-t1)) holds without being used; a
    centred constant gives 0."""
    x = synth.iid_exp_centered(60, 4)
    c = oracle.c5_hyper(x, 2)
    for perm in [(1, 0, 2, 3), (0, 2, 1, 3), (0, 1, 3, 2), (3, 2, 1, 0)]:
        assert np.max(np.abs(c - c.transpose(perm))) < 1e-14 * np.max(np.abs(c))
    M = 2
    t = np.arange(-M, M + 1)
    a, b, cc, d = np.meshgrid(t, t, t, t, indexing="ij")
    ok = (np.abs(b - a) <= M) & (np.abs(cc - a) <= M) & (np.abs(d - a) <= M)
    lhs = c[ok]
    rhs = c[(-a)[ok] + M, (b - a)[ok] + M, (cc - a)[ok] + M, (d - a)[ok] + M]
    assert np.max(np.abs(lhs - rhs)) < 1e-14 * np.max(np.abs(c))
    assert np.max(np.abs(oracle.c5_hyper(np.full(30, 2.5), 1))) < 1e-12


def test_window5_hand_values():
    """Product of d over the ten differences of {0, t1, t2, t3, t4}, M = 4:
    d(0) = 1, d(1) = 1 - 6/16 + 6/64 = 0.71875, d(2) = 0.25 (r = 1/2:
    1 - 6/4 + 6/8), d(3) = 2 (1/4)^3 = 0.03125, d(4) = 0."""
    w = oracle.window5(4)
    d = {0: 1.0, 1: 0.71875, 2: 0.25, 3: 0.03125, 4: 0.0}
    at = lambda *t: w[tuple(np.asarray(t) + 4)]
    # (1, 1, 0, 0): differences 1,1,0,0, 0,1,1, 1,1, 0
    assert abs(at(1, 1, 0, 0) - d[1] ** 6) < 1e-15
    # (1, 2, 0, -1): offsets {0,1,2,0,-1}: |diffs| = 1,2,0,1, 1,1,2, 2,3, 1
    assert abs(at(1, 2, 0, -1) - d[1] ** 5 * d[2] ** 3 * d[3] * d[0]) < 1e-15
    assert at(4, 0, 0, 0) == 0.0


def test_spectrum5_fold_and_symmetry():
    """With N = 2M the folded 4-D DFT equals the direct sum over every lag
    (aliases included) at sampled frequencies; the spectrum is Hermitian and
    symmetric under permutations of (k1..k4)."""
    x = synth.iid_exp_centered(70, 6)
    M, N = 2, 4
    c, Q = oracle.spectrum5(x, M, N)
    cw = c * oracle.window5(M)
    lag = np.arange(-M, M + 1)
    for k in [(0, 0, 0, 0), (1, 2, 3, 0), (3, 3, 1, 2)]:
        ph = np.exp(-2j * np.pi * (k[0] * lag[:, None, None, None] + k[1] * lag[None, :, None, None]
                                   + k[2] * lag[None, None, :, None]
                                   + k[3] * lag[None, None, None, :]) / N)
        assert abs(np.sum(cw * ph) - Q[k]) < 1e-12 * np.max(np.abs(Q))
    kk = np.arange(N)
    Qm = Q[np.ix_(*[(-kk) % N] * 4)]
    assert np.max(np.abs(Q - np.conj(Qm))) < 1e-12 * np.max(np.abs(Q))
    assert np.max(np.abs(Q - Q.transpose(1, 0, 3, 2))) < 1e-12 * np.max(np.abs(Q))
