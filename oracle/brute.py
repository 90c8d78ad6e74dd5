"""Pure-Python literal loops for tiny inputs (test infrastructure only).

A second, independent spelling of the oracle's sums: it tests every index of
every term against the record bounds instead of precomputing the valid t
range, so an off-by-one in the C core's range shows up as a mismatch.  It is
meant for n of a few dozen samples.
"""
from __future__ import annotations


def _inrange(n, *idx):
    return all(0 <= i < n for i in idx)


def center(x):
    n = len(x)
    mu = sum(x) / n
    return [v - mu for v in x]


def c3(x, w1, w2):
    n = len(x)
    s = 0.0
    for t in range(-2 * n, 2 * n):
        if _inrange(n, t, t + w1, t + w2):
            s += x[t] * x[t + w1] * x[t + w2]
    return s / n


def c2(x, d):
    n = len(x)
    s = 0.0
    for t in range(-2 * n, 2 * n):
        if _inrange(n, t, t + d):
            s += x[t] * x[t + d]
    return s / n


def m4(x, t1, t2, t3):
    n = len(x)
    s = 0.0
    for t in range(-3 * n, 3 * n):
        if _inrange(n, t, t + t1, t + t2, t + t3):
            s += x[t] * x[t + t1] * x[t + t2] * x[t + t3]
    return s / n


def c4(x, t1, t2, t3):
    return (m4(x, t1, t2, t3) - c2(x, t1) * c2(x, t3 - t2)
            - c2(x, t2) * c2(x, t3 - t1) - c2(x, t3) * c2(x, t2 - t1))


def m5(x, t1, t2, t3, t4):
    n = len(x)
    s = 0.0
    for t in range(-3 * n, 3 * n):
        if _inrange(n, t, t + t1, t + t2, t + t3, t + t4):
            s += x[t] * x[t + t1] * x[t + t2] * x[t + t3] * x[t + t4]
    return s / n


def c5(x, t1, t2, t3, t4):
    """m5 minus c2 * c3 over the ten ways to split the offsets
    (0, t1, t2, t3, t4) into a pair and a triple, listed one by one."""
    o = (0, t1, t2, t3, t4)
    pairs = ((0, 1), (0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 4))
    v = m5(x, t1, t2, t3, t4)
    for j, k in pairs:
        p, q, r = [o[i] for i in range(5) if i not in (j, k)]
        v -= c2(x, o[k] - o[j]) * c3(x, q - p, r - p)
    return v
