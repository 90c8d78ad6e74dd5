"""FP64 CPU oracle for the smoothed sample bispectrum / trispectrum.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1805_11775_amd``) and never imports it;
the product path never calls into it.

What it computes, and the passages it follows (arXiv:1805.11775):

* mean removal -- Section 1, Algorithm DBS's per-part mean removal (subtract the mean of a
  part), with the whole record as one part (Section 4.1 uses K = 1);
* the third and fourth sample cumulants -- Section 1 "Problem Statement"
  (moments of order k, cumulants as functions of moments, time averages in
  place of ensemble averages); the brute-force sums live in
  ``hos_oracle.c``;
* the spectra as Fourier transforms of the cumulants -- Section 1 (the
  bispectrum transforms the third cumulant, the trispectrum the fourth),
  with the DFT sign of Algorithm DBS's part DFT (exp(-j 2 pi u k / M),
  unnormalised);
* the principal domain 0 <= k2 <= k1, k1 + k2 < N/2 -- Algorithm DBS's raw bispectrum.

Where the paper is silent (normalisation 1/n, lag-window shape, output
region, loss), each function below states the reading it uses.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C core with gcc (plain -O2, no fast-math reassociation)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.or_center.argtypes = [dp, i64, dp]
        lib.or_c3_at.argtypes = [dp, i64, ip, ip, i64, dp]
        lib.or_c3_square.argtypes = [dp, i64, i32, dp]
        lib.or_c2.argtypes = [dp, i64, i32, dp]
        lib.or_m4_at.argtypes = [dp, i64, ip, ip, ip, i64, dp]
        lib.or_c4_at.argtypes = [dp, i64, ip, ip, ip, i64, dp]
        lib.or_c4_cube.argtypes = [dp, i64, i32, dp]
        lib.or_m5_at.argtypes = [dp, i64, ip, ip, ip, ip, i64, dp]
        lib.or_c5_at.argtypes = [dp, i64, ip, ip, ip, ip, i64, dp]
        lib.or_c5_hyper.argtypes = [dp, i64, i32, dp]
        lib.or_c3_grad.argtypes = [dp, i64, i32, dp, dp]
        lib.or_c3_grad_at.argtypes = [dp, i64, i32, dp, ctypes.POINTER(ctypes.c_int64), i64,
                                      dp]
        for f in (lib.or_center, lib.or_c3_at, lib.or_c3_square, lib.or_c2,
                  lib.or_m4_at, lib.or_c4_at, lib.or_c4_cube, lib.or_c3_grad,
                  lib.or_c3_grad_at, lib.or_m5_at, lib.or_c5_at, lib.or_c5_hyper):
            f.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# --------------------------------------------------------------------------
# Stage 1: mean removal (Algorithm DBS's per-part mean removal with one part, K = 1).
# --------------------------------------------------------------------------
def center(x) -> np.ndarray:
    """x - mean(x) in FP64 (input widened exactly from float32 if needed)."""
    x = _f64(x)
    out = np.empty_like(x)
    _load().or_center(_dp(x), x.size, _dp(out))
    return out


def _prep(x, centered: bool) -> np.ndarray:
    return center(x) if centered else _f64(x)


# --------------------------------------------------------------------------
# Stage 2: sample cumulants (Section 1, Problem Statement), brute force.
# --------------------------------------------------------------------------
def c3_at(x, w1, w2, centered: bool = True) -> np.ndarray:
    """c3(w1[k], w2[k]) = (1/n) sum_t x_t x_{t+w1} x_{t+w2}, any lags."""
    xt = _prep(x, centered)
    w1 = np.ascontiguousarray(np.asarray(w1, dtype=np.int32).ravel())
    w2 = np.ascontiguousarray(np.asarray(w2, dtype=np.int32).ravel())
    out = np.empty(w1.size, dtype=np.float64)
    _load().or_c3_at(_dp(xt), xt.size, _ip(w1), _ip(w2), w1.size, _dp(out))
    return out


def c3_square(x, M: int, centered: bool = True) -> np.ndarray:
    """c3 at every lag of the square |w1|, |w2| <= M; [w1+M, w2+M]."""
    xt = _prep(x, centered)
    side = 2 * M + 1
    out = np.empty((side, side), dtype=np.float64)
    _load().or_c3_square(_dp(xt), xt.size, int(M), _dp(out))
    return out


def span3(M: int) -> np.ndarray:
    """max(0,w1,w2) - min(0,w1,w2) over the square, [w1+M, w2+M]."""
    w = np.arange(-M, M + 1)
    w1, w2 = np.meshgrid(w, w, indexing="ij")
    return np.maximum(np.maximum(0, w1), w2) - np.minimum(np.minimum(0, w1), w2)


def c3_hexagon(x, M: int, centered: bool = True) -> np.ndarray:
    """c3 on the hexagon |w1|,|w2|,|w1-w2| <= M, zero on the two corners.

    Output-region reading: the lags requested are |w| <= M; the hexagon is
    the set of those lags whose whole six-fold symmetry orbit stays inside
    the square, so an estimate over it keeps the symmetries of c3 (and B
    those of the bispectrum).  The corner lags (|w1 - w2| > M) are outside
    it and set to 0; the Parzen window W3 vanishes there in any case.
    """
    c = c3_square(x, M, centered)
    c[span3(M) > M] = 0.0
    return c


def c2(x, M: int, centered: bool = True) -> np.ndarray:
    """c2(d) = (1/n) sum_t x_t x_{t+d}, d = 0..M."""
    xt = _prep(x, centered)
    out = np.empty(M + 1, dtype=np.float64)
    _load().or_c2(_dp(xt), xt.size, int(M), _dp(out))
    return out


def m4_at(x, t1, t2, t3, centered: bool = True) -> np.ndarray:
    xt = _prep(x, centered)
    t1, t2, t3 = (np.ascontiguousarray(np.asarray(t, dtype=np.int32).ravel())
                  for t in (t1, t2, t3))
    out = np.empty(t1.size, dtype=np.float64)
    _load().or_m4_at(_dp(xt), xt.size, _ip(t1), _ip(t2), _ip(t3), t1.size,
                     _dp(out))
    return out


def c4_at(x, t1, t2, t3, centered: bool = True) -> np.ndarray:
    """c4 = m4 - (three products of c2), at arbitrary lag triples."""
    xt = _prep(x, centered)
    t1, t2, t3 = (np.ascontiguousarray(np.asarray(t, dtype=np.int32).ravel())
                  for t in (t1, t2, t3))
    out = np.empty(t1.size, dtype=np.float64)
    _load().or_c4_at(_dp(xt), xt.size, _ip(t1), _ip(t2), _ip(t3), t1.size,
                     _dp(out))
    return out


def c4_cube(x, M: int, centered: bool = True) -> np.ndarray:
    """c4 at every lag of the cube |t_i| <= M; [t1+M, t2+M, t3+M]."""
    xt = _prep(x, centered)
    S = 2 * M + 1
    out = np.empty((S, S, S), dtype=np.float64)
    _load().or_c4_cube(_dp(xt), xt.size, int(M), _dp(out))
    return out


def span4(M: int) -> np.ndarray:
    """max - min of {0, t1, t2, t3} over the cube."""
    t = np.arange(-M, M + 1)
    t1, t2, t3 = np.meshgrid(t, t, t, indexing="ij")
    mx = np.maximum(np.maximum(np.maximum(0, t1), t2), t3)
    mn = np.minimum(np.minimum(np.minimum(0, t1), t2), t3)
    return mx - mn


def c4_support(x, M: int, centered: bool = True) -> np.ndarray:
    """c4 on {span(0,t1,t2,t3) <= M}, zero elsewhere in the cube: the lags
    of the cube whose whole 24-fold symmetry orbit stays inside the cube
    (the hexagon's counterpart one order up)."""
    c = c4_cube(x, M, centered)
    c[span4(M) > M] = 0.0
    return c


def _quad(t1, t2, t3, t4):
    return tuple(np.ascontiguousarray(np.asarray(t, dtype=np.int32).ravel())
                 for t in (t1, t2, t3, t4))


def m5_at(x, t1, t2, t3, t4, centered: bool = True) -> np.ndarray:
    """Fifth-order sample moment (1/n) sum_t x_t x_{t+t1} .. x_{t+t4}."""
    xt = _prep(x, centered)
    t1, t2, t3, t4 = _quad(t1, t2, t3, t4)
    out = np.empty(t1.size, dtype=np.float64)
    _load().or_m5_at(_dp(xt), xt.size, _ip(t1), _ip(t2), _ip(t3), _ip(t4), t1.size,
                     _dp(out))
    return out


def c5_at(x, t1, t2, t3, t4, centered: bool = True) -> np.ndarray:
    """c5 = m5 - (ten products c2 * m3 over the pair / triple partitions of
    the five offsets), at arbitrary lag quadruples (Section 1: cumulants as
    functions of moments, the order-5 case of the moment-to-cumulant
    relation for zero-mean variables)."""
    xt = _prep(x, centered)
    t1, t2, t3, t4 = _quad(t1, t2, t3, t4)
    out = np.empty(t1.size, dtype=np.float64)
    _load().or_c5_at(_dp(xt), xt.size, _ip(t1), _ip(t2), _ip(t3), _ip(t4), t1.size,
                     _dp(out))
    return out


def c5_hyper(x, M: int, centered: bool = True) -> np.ndarray:
    """c5 at every lag of the hypercube |t_i| <= M; [t1+M, t2+M, t3+M, t4+M]."""
    xt = _prep(x, centered)
    S = 2 * M + 1
    out = np.empty((S, S, S, S), dtype=np.float64)
    _load().or_c5_hyper(_dp(xt), xt.size, int(M), _dp(out))
    return out


def span5(M: int) -> np.ndarray:
    """max - min of {0, t1, t2, t3, t4} over the hypercube."""
    t = np.arange(-M, M + 1)
    g = np.meshgrid(t, t, t, t, indexing="ij")
    mx = np.maximum.reduce([np.zeros_like(g[0])] + list(g))
    mn = np.minimum.reduce([np.zeros_like(g[0])] + list(g))
    return mx - mn


def c5_support(x, M: int, centered: bool = True) -> np.ndarray:
    """c5 on {span(0,t1,t2,t3,t4) <= M}, zero elsewhere in the hypercube."""
    c = c5_hyper(x, M, centered)
    c[span5(M) > M] = 0.0
    return c


# --------------------------------------------------------------------------
# Stage 3: lag window (the paper smooths in frequency with a box; the
# workloads use the Parzen lag window instead -- a reading).
# --------------------------------------------------------------------------
def parzen(m, L: int) -> np.ndarray:
    """Parzen lag window d(m) with scale L: 1-6r^2+6r^3 (r<=1/2),
    2(1-r)^3 (1/2<r<=1), 0 beyond; r = |m|/L.  At L = 0 (maximum lag 0)
    r is undefined; the limit L -> 0+ gives d(0) = 1 and d(m != 0) = 0."""
    m = np.asarray(m, dtype=np.float64)
    if L == 0:
        return np.where(m == 0, 1.0, 0.0)
    r = np.abs(m) / float(L)
    return np.where(r <= 0.5, 1.0 - 6.0 * r ** 2 + 6.0 * r ** 3,
                    np.where(r <= 1.0, 2.0 * (1.0 - r) ** 3, 0.0))


def window3(M: int, kind: str = "parzen") -> np.ndarray:
    """W3(w1,w2) = d(w1) d(w2) d(w1-w2) over the square, scale L = M;
    kind "separable": d(w1) d(w2); "none": 1."""
    w = np.arange(-M, M + 1)
    w1, w2 = np.meshgrid(w, w, indexing="ij")
    if kind == "none":
        return np.ones_like(w1, dtype=np.float64)
    if kind == "separable":
        return parzen(w1, M) * parzen(w2, M)
    return parzen(w1, M) * parzen(w2, M) * parzen(w1 - w2, M)


def window4(M: int, kind: str = "parzen") -> np.ndarray:
    """Product of d over the six pairwise differences of {0,t1,t2,t3};
    kind "separable": d(t1) d(t2) d(t3); "none": 1."""
    t = np.arange(-M, M + 1)
    t1, t2, t3 = np.meshgrid(t, t, t, indexing="ij")
    if kind == "none":
        return np.ones_like(t1, dtype=np.float64)
    d = lambda m: parzen(m, M)
    if kind == "separable":
        return d(t1) * d(t2) * d(t3)
    return d(t1) * d(t2) * d(t3) * d(t2 - t1) * d(t3 - t1) * d(t3 - t2)


def window5(M: int, kind: str = "parzen") -> np.ndarray:
    """Product of d over the ten pairwise differences of {0,t1,t2,t3,t4};
    kind "separable": d(t1) d(t2) d(t3) d(t4); "none": 1."""
    t = np.arange(-M, M + 1)
    g = np.meshgrid(t, t, t, t, indexing="ij")
    if kind == "none":
        return np.ones_like(g[0], dtype=np.float64)
    d = lambda m: parzen(m, M)
    if kind == "separable":
        return d(g[0]) * d(g[1]) * d(g[2]) * d(g[3])
    pts = [np.zeros_like(g[0])] + list(g)
    w = np.ones_like(g[0], dtype=np.float64)
    for j in range(5):
        for k in range(j + 1, 5):
            w = w * d(pts[k] - pts[j])
    return w


# --------------------------------------------------------------------------
# Stage 4: the DFT (Section 1: spectra are Fourier transforms of cumulants;
# sign and normalisation of Algorithm DBS's part DFT).
# --------------------------------------------------------------------------
def place_circular(c: np.ndarray, M: int, N: int) -> np.ndarray:
    """Fold a lag-domain array on [-M, M]^d onto the N^d DFT grid: the value
    at index m is the sum of c over all lags w with w = m (mod N).  Its DFT is
    then exactly sum_w c(w) exp(-2 pi i <k, w> / N) at the grid frequencies."""
    d = c.ndim
    out = np.zeros((N,) * d, dtype=np.float64)
    idx = np.arange(-M, M + 1) % N
    np.add.at(out, np.ix_(*([idx] * d)), c)
    return out


def bispectrum(x, M: int, nfft: int, window: str = "parzen",
               centered: bool = True, full_square: bool = False):
    """(c3 over the lag region, B = 2D DFT of the windowed c3 on an N x N grid).

    B(k1,k2) = sum_w W3(w) c3(w) exp(-2 pi i (k1 w1 + k2 w2)/N), unshifted
    frequency order, no normalisation.  The lag region is the hexagon (the
    lags of the square whose whole six-fold orbit stays in the square, zero
    on the two corners) or, with ``full_square``, every lag |w1|, |w2| <= M
    (Section 1, Problem Statement: the sample cumulant at every lag up to
    the maximum lag).
    """
    sq = c3_square(x, M, centered)
    c = sq if full_square else np.where(span3(M) > M, 0.0, sq)
    # B transforms the windowed sample cumulant over every lag of the square
    # (Section 1, Problem Statement); the Parzen product W3 vanishes on the
    # corners, the separable window and no window do not
    B = np.fft.fft2(place_circular(sq * window3(M, window), M, nfft))
    return c, B


def spectrum5(x, M: int, nfft: int, window: str = "parzen", centered: bool = True):
    """(c5 on its support, Q = 4D DFT of the windowed c5 on an N^4 grid): the
    order-5 member of the family (the paper's k-th order spectrum)."""
    hyper = c5_hyper(x, M, centered)
    c = np.where(span5(M) > M, 0.0, hyper)
    Q = np.fft.fftn(place_circular(hyper * window5(M, window), M, nfft))
    return c, Q


def trispectrum(x, M: int, nfft: int, window: str = "parzen",
                centered: bool = True):
    """(c4 on its support, T = 3D DFT of the windowed c4 on an N^3 grid)."""
    cube = c4_cube(x, M, centered)
    c = np.where(span4(M) > M, 0.0, cube)
    # T transforms the windowed sample cumulant over the whole cube; the
    # Parzen product over the six differences vanishes where the span
    # exceeds M, the separable window and no window do not
    T = np.fft.fftn(place_circular(cube * window4(M, window), M, nfft))
    return c, T


def bispectrum_segments(x, P: int, M: int, nfft: int, window: str = "parzen",
                        centered: bool = True):
    """Segment averaging for the indirect estimator: Algorithm DBS's split
    into parts, per-part mean removal and average over parts, around the
    cumulant.  K = floor(n / P) segments of P consecutive samples (trailing
    samples unused), each centred on its own mean, the third cumulant of
    each (the single-series estimator above, with the segment as the
    record), their average over the segments, then
    the window and the DFT as in ``bispectrum``.  Returns (c3, B)."""
    x = _f64(x)
    K = x.size // P
    c = np.zeros((2 * M + 1, 2 * M + 1))
    for i in range(K):
        c += c3_square(x[i * P:(i + 1) * P], M, centered)
    c /= K
    B = np.fft.fft2(place_circular(c * window3(M, window), M, nfft))
    c[span3(M) > M] = 0.0
    return c, B


# --------------------------------------------------------------------------
# Principal domain (Algorithm DBS's raw bispectrum) and the matching loss.
# --------------------------------------------------------------------------
def pd_indices(N: int):
    """(k1, k2) of the principal domain 0 <= k2 <= k1, k1 + k2 < N/2,
    in row-major (k1, then k2) order."""
    k1, k2 = [], []
    for a in range(N):
        for b in range(a + 1):
            if 2 * (a + b) < N:
                k1.append(a)
                k2.append(b)
    return np.asarray(k1, dtype=np.int64), np.asarray(k2, dtype=np.int64)


def bispectrum_pd(x, M: int, nfft: int, window: str = "parzen", centered: bool = True):
    """B at the principal-domain frequencies, in ``pd_indices`` order."""
    _, B = bispectrum(x, M, nfft, window, centered)
    k1, k2 = pd_indices(nfft)
    return B[k1, k2]


def bispectrum_loss(X, M: int, nfft: int, target_pd, window: str = "parzen"):
    """L = sum over series and principal-domain frequencies of
    |B(x_b)(k) - target(k)|^2; X is (batch, n) or (n,)."""
    X = np.atleast_2d(_f64(X))
    t = np.asarray(target_pd, dtype=np.complex128)
    return float(sum(np.sum(np.abs(bispectrum_pd(xb, M, nfft, window) - t) ** 2)
                     for xb in X))


def loss_weight(x, M: int, nfft: int, target_pd, window: str = "parzen") -> np.ndarray:
    """G(w) = dL/dc3(w) over the square for one series: with R = B - target
    on the principal domain and B = sum_w W3(w) c3(w) e^{-2 pi i <k,w>/N},
    dL/dc3(w) = 2 W3(w) Re sum_k R_k e^{+2 pi i <k,w>/N}, over every lag of
    the square (the Parzen product W3 makes it 0 on the corners)."""
    k1, k2 = pd_indices(nfft)
    R = bispectrum_pd(x, M, nfft, window) - np.asarray(target_pd, dtype=np.complex128)
    Rm = np.zeros((nfft, nfft), dtype=np.complex128)
    Rm[k1, k2] = R
    w = np.arange(-M, M + 1)
    E = np.exp(2j * np.pi * np.outer(np.arange(nfft), w) / nfft)   # E[k, w]
    S = E.T @ Rm @ E                                               # sum_k R_k e^{+i..}
    return 2.0 * window3(M, window) * S.real


def bispectrum_loss_grad(X, M: int, nfft: int, target_pd, window: str = "parzen",
                         dL: float = 1.0) -> np.ndarray:
    """dL/dx for every series (same shape as X): the chain rule through
    c3 (``or_c3_grad``) and through the mean removal, d/dx_j = d/dx~_j minus
    the mean over j of d/dx~."""
    X2 = np.atleast_2d(_f64(X))
    out = np.empty_like(X2)
    for b, xb in enumerate(X2):
        G = np.ascontiguousarray(loss_weight(xb, M, nfft, target_pd, window))
        xt = center(xb)
        g = np.empty_like(xt)
        _load().or_c3_grad(_dp(xt), xt.size, int(M), _dp(G), _dp(g))
        out[b] = dL * (g - np.mean(g))
    return out.reshape(np.shape(X))


def loss_grad_at(x, M: int, nfft: int, target_pd, idx, window: str = "parzen") -> np.ndarray:
    """dL/dx~_j (before the mean-removal term) of one series at the indices
    ``idx``; differences of these equal differences of dL/dx."""
    G = np.ascontiguousarray(loss_weight(x, M, nfft, target_pd, window))
    xt = center(x)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.size, dtype=np.float64)
    _load().or_c3_grad_at(_dp(xt), xt.size, int(M), _dp(G),
                          idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size, _dp(out))
    return out


# --------------------------------------------------------------------------
# The paper's direct method (Algorithm DBS), in its own step order.
# Readings: K = floor(n / P) parts of P samples (trailing samples unused);
# the raw bispectrum uses F(k1) F(k2) conj(F(k1+k2)) / P (the conjugate the
# printed raw bispectrum lacks); the M3 x M3 box takes exactly M3 offsets per axis,
# n in [-floor(M3/2), M3 - 1 - floor(M3/2)], indices modulo P.
# --------------------------------------------------------------------------
def dbs_raw(part) -> np.ndarray:
    """Algorithm DBS for one part: mean removed, P-point DFT, and the raw
    bispectrum C(k1, k2) = F(k1) F(k2) conj(F(k1 + k2)) / P on the whole
    P x P grid (indices modulo P)."""
    xp = _f64(part)
    xp = xp - np.mean(xp)
    P = xp.size
    F = np.fft.fft(xp)
    k = np.arange(P)
    return F[:, None] * F[None, :] * np.conj(F[(k[:, None] + k[None, :]) % P]) / P


def dbs_smooth(C, M3: int) -> np.ndarray:
    """Algorithm DBS's box smoothing: average of C over the M3 x M3 box of offsets around each
    point, indices modulo the grid size (written as the double sum)."""
    lo = M3 // 2
    out = np.zeros_like(C)
    for n1 in range(-lo, M3 - lo):
        for n2 in range(-lo, M3 - lo):
            out += np.roll(np.roll(C, -n1, axis=0), -n2, axis=1)
    return out / float(M3 * M3)


def dbs(x, P: int, M3: int) -> np.ndarray:
    """Algorithm DBS: partition, per part raw bispectrum and smoothing, then
    the average over parts; returned on the principal domain (pd_indices(P)
    order)."""
    x = _f64(x)
    K = x.size // P
    acc = np.zeros((P, P), dtype=np.complex128)
    for i in range(K):
        acc += dbs_smooth(dbs_raw(x[i * P:(i + 1) * P]), M3)
    k1, k2 = pd_indices(P)
    return (acc / K)[k1, k2]


def c3_circular(part) -> np.ndarray:
    """(1/P) sum_t x_t x_{(t+w1) mod P} x_{(t+w2) mod P} for the mean-removed
    part, every (w1, w2) in [0, P)^2, by brute force (pins dbs_raw)."""
    xp = _f64(part)
    xp = xp - np.mean(xp)
    P = xp.size
    out = np.empty((P, P))
    t = np.arange(P)
    for w1 in range(P):
        for w2 in range(P):
            out[w1, w2] = np.sum(xp * xp[(t + w1) % P] * xp[(t + w2) % P]) / P
    return out


def dbs_at(x, P: int, M3: int, k1, k2) -> np.ndarray:
    """Algorithm DBS at chosen frequencies only: for each (k1, k2), the
    M3 x M3 box of raw part bispectra written out as an explicit double sum
    (indices modulo P), averaged over the parts.  For outputs of grids too
    large for ``dbs``."""
    x = _f64(x)
    K = x.size // P
    k1 = np.atleast_1d(np.asarray(k1, dtype=np.int64))
    k2 = np.atleast_1d(np.asarray(k2, dtype=np.int64))
    lo = M3 // 2
    off = np.arange(-lo, M3 - lo)
    out = np.zeros(k1.size, dtype=np.complex128)
    for i in range(K):
        xp = x[i * P:(i + 1) * P]
        F = np.fft.fft(xp - np.mean(xp))
        for j in range(k1.size):
            a = (k1[j] + off) % P
            b = (k2[j] + off) % P
            raw = F[a][:, None] * F[b][None, :] * np.conj(F[(a[:, None] + b[None, :]) % P])
            out[j] += np.sum(raw) / P
    return out / (K * float(M3 * M3))
