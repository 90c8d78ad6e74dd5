"""Seeded synthetic input series for the bispectrum / trispectrum workloads.

This module only draws input data.  It holds none of the estimator's
arithmetic (no centering, no cumulants, no windows, no transforms), so both
the FP64 CPU oracle and the GPU path may use it without sharing any of the
method's code.

Every generator takes an explicit integer seed and returns float64 numpy
arrays; callers cast to float32 where a workload is specified in float32
(the cast is part of the workload definition, not of the method).

Recipes (the paper's own data generators are not available, so these
stand in for its workloads, at the sizes of interest in its experiments):

* ``iid_exp_centered``  Exp(1) - 1, i.i.d.  (third cumulant 2, fourth 6)
* ``iid_gauss``         N(0, 1), i.i.d.     (all cumulants above 2 vanish)
* ``quadratic_process`` x_t = e_t + b e_{t-1} e_{t-2}, e ~ N(0,1), b = 0.5
* ``cubic_process``     x_t = e_t + b e_{t-1} e_{t-2} e_{t-3}, b = 0.4
* ``batched_series``    many series of uneven length and maximum lag

The innovations e are drawn for t = -p .. n-1 (p = process order), so the
output x_0 .. x_{n-1} is stationary from its first sample.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 180511775

# Maximum-lag choices and length range of the batched workload.
BATCH_M_CHOICES = (32, 64, 128, 256)
BATCH_N_RANGE = (1024, 65536)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def iid_exp_centered(n: int, seed: int) -> np.ndarray:
    """n i.i.d. samples of Exp(1) - 1."""
    return _rng(seed).exponential(1.0, size=int(n)) - 1.0


def iid_gauss(n: int, seed: int) -> np.ndarray:
    """n i.i.d. standard normal samples."""
    return _rng(seed).standard_normal(int(n))


def quadratic_process(n: int, seed: int, b: float = 0.5) -> np.ndarray:
    """x_t = e_t + b e_{t-1} e_{t-2} for t = 0..n-1 with e ~ N(0,1)."""
    n = int(n)
    e = _rng(seed).standard_normal(n + 2)  # e[k] is e_{k-2}
    return e[2:] + b * e[1:-1] * e[:-2]


def cubic_process(n: int, seed: int, b: float = 0.4) -> np.ndarray:
    """x_t = e_t + b e_{t-1} e_{t-2} e_{t-3} for t = 0..n-1 with e ~ N(0,1)."""
    n = int(n)
    e = _rng(seed).standard_normal(n + 3)  # e[k] is e_{k-3}
    return e[3:] + b * e[2:-1] * e[1:-2] * e[:-3]


def quartic_process(n: int, seed: int, b: float = 0.3) -> np.ndarray:
    """x_t = e_t + b e_{t-1} e_{t-2} e_{t-3} e_{t-4} for t = 0..n-1, e ~ N(0,1):
    its fifth cumulant is b at the offsets {0, 1, 2, 3, 4} (up to order b^3)."""
    n = int(n)
    e = _rng(seed).standard_normal(n + 4)  # e[k] is e_{k-4}
    return e[4:] + b * e[3:-1] * e[2:-2] * e[1:-3] * e[:-4]


def batched_series(batch: int, seed: int, n_range=BATCH_N_RANGE,
                   m_choices=BATCH_M_CHOICES):
    """Return (list of float64 series, lengths, max lags) for a batch.

    Even indices are N(0,1) i.i.d., odd indices centred Exp(1) i.i.d.;
    lengths are integer-uniform on ``n_range`` (inclusive) and the maximum
    lag is uniform over ``m_choices``.  Each series has its own stream
    spawned from ``seed`` so a subset can be regenerated on its own.
    """
    ss = np.random.SeedSequence(int(seed))
    meta = _rng(seed)
    lo, hi = int(n_range[0]), int(n_range[1])
    lengths = meta.integers(lo, hi + 1, size=int(batch))
    lags = meta.choice(np.asarray(m_choices, dtype=np.int64), size=int(batch))
    children = ss.spawn(int(batch))
    out = []
    for k in range(int(batch)):
        g = np.random.Generator(np.random.PCG64(children[k]))
        nk = int(lengths[k])
        if k % 2 == 0:
            out.append(g.standard_normal(nk))
        else:
            out.append(g.exponential(1.0, size=nk) - 1.0)
    return out, lengths.astype(np.int64), lags.astype(np.int64)


def batched_one(batch: int, seed: int, k: int, n_range=BATCH_N_RANGE,
                m_choices=BATCH_M_CHOICES):
    """Series k of ``batched_series(batch, seed)`` without drawing the rest."""
    ss = np.random.SeedSequence(int(seed))
    meta = _rng(seed)
    lo, hi = int(n_range[0]), int(n_range[1])
    lengths = meta.integers(lo, hi + 1, size=int(batch))
    lags = meta.choice(np.asarray(m_choices, dtype=np.int64), size=int(batch))
    child = ss.spawn(int(batch))[k]
    g = np.random.Generator(np.random.PCG64(child))
    nk = int(lengths[k])
    x = g.standard_normal(nk) if k % 2 == 0 else g.exponential(1.0, size=nk) - 1.0
    return x, int(lengths[k]), int(lags[k])


# Named workloads: (generator, n, seed, dtype).  Sizes follow the workload
# definitions of the bispectrum/trispectrum benchmarks.
def workload_small_bispectrum():
    """n=2048 float64 centred Exp(1), maximum lag 64, 128-point DFT."""
    return iid_exp_centered(2048, SEED_BASE + 1), dict(M=64, nfft=128)


def workload_long_bispectrum(n: int = 1 << 20):
    """n=2^20 float32 quadratic process, maximum lag 512, 1024-point DFT."""
    x = quadratic_process(n, SEED_BASE + 2).astype(np.float32)
    return x, dict(M=512, nfft=1024)


def workload_trispectrum(n: int = 1 << 18):
    """n=2^18 float32 cubic process, maximum lag 48, 96^3 DFT."""
    x = cubic_process(n, SEED_BASE + 3).astype(np.float32)
    return x, dict(M=48, nfft=96)


def workload_batched(batch: int = 4096):
    """4096 series: n uniform in [1024, 65536], M uniform over {32,64,128,256},
    even index N(0,1), odd index Exp(1) - 1 (float64 here; cast to float32
    for the benchmark)."""
    return batched_series(batch, SEED_BASE + 4)


def workload_loss(batch: int = 64, n: int = 65536):
    """(X, target series, config): X is `batch` i.i.d. N(0,1) float32 series
    of length n (one spawned stream each); the target spectrum comes from a
    quadratic-process series of the same length; M = 256, 512-point DFT."""
    ss = np.random.SeedSequence(SEED_BASE + 5)
    X = np.stack([np.random.Generator(np.random.PCG64(c)).standard_normal(int(n))
                  for c in ss.spawn(int(batch))]).astype(np.float32)
    target = quadratic_process(n, SEED_BASE + 6)
    return X, target, dict(M=256, nfft=512)


def workload_dbs(n: int = 1 << 16):
    """Direct method: one float32 quadratic-process series of 2^16 samples
    taken as a single part (K = 1, P = n), smoothed over a 1023 x 1023 box
    (the window lengths of the paper's timing table grow by about 1.54 per
    doubling of n, which puts n = 2^16 near 1020)."""
    x = quadratic_process(n, SEED_BASE + 7).astype(np.float32)
    return x, dict(P=int(n), M3=1023)


def workload_segments(n: int = 1 << 20):
    """Segment averaging: the long bispectrum's series (n = 2^20 float32
    quadratic process) cut into 16 segments of 65536 samples, maximum lag
    512, 1024-point DFT."""
    x, cfg = workload_long_bispectrum(n)
    return x, dict(P=n // 16, M=cfg["M"], nfft=cfg["nfft"])


def workload_cumulant5(n: int = 1 << 18):
    """Order five: n = 2^18 float32 quartic process, maximum lag 24, 48^4 DFT."""
    x = quartic_process(n, SEED_BASE + 8).astype(np.float32)
    return x, dict(M=24, nfft=48)


def workload_streamed(n: int = 1 << 26):
    """A record held in host memory: n = 2^26 float32 quadratic process
    (64 times the long bispectrum's series), maximum lag 512, 1024-point
    DFT, read in pieces of 2^22 samples."""
    x = quadratic_process(n, SEED_BASE + 9).astype(np.float32)
    return x, dict(M=512, nfft=1024, piece=1 << 22)
