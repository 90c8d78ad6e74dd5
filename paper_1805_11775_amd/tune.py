"""Autotuner for the batched contraction's tile shape.

For every maximum lag M of a batch the contraction can run on tiles of
2 x 2 or 4 x 4 matrix-core blocks (split paths; the FP32 path has 4 x 4
tiles only).  Small tiles waste less of the triangle at small M, large tiles
reuse each product row across more columns.  ``tune`` times both on the
device: for each M it builds a synthetic batch of series with lengths
spread over [n_lo, n_hi], runs the batched bispectrum under each choice,
keeps the median over several calls of the contraction stage's time (HIP
events around that stage alone; the other stages do not depend on the
tile) and picks the fastest.  The result (and its timings) can be saved as JSON and
passed to ``BatchPlan(..., tile=choices)``.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import BatchPlan, bispectrum_batched_timed

CANDIDATES = {"fp32": (4,), "split_fp16": (2, 4), "split_bf16": (2, 4)}


def _batch(M, series, n_lo, n_hi, seed):
    rng = np.random.default_rng(seed)
    n = np.maximum(rng.integers(n_lo, n_hi + 1, size=series), M + 2)
    x = rng.standard_normal(int(np.sum(n))).astype(np.float32)
    return n, x


def tune(Ms, path="split_fp16", n_lo=1024, n_hi=65536, series=128, reps=5, seed=1,
         cache=None, device="cuda"):
    """Returns {"path": path, "choices": {M: tile}, "ms": {M: {tile: median ms}}};
    written to ``cache`` (JSON) when given."""
    import torch
    out = {"path": path, "measure": "contraction stage, median ms",
           "n_range": [int(n_lo), int(n_hi)], "series": int(series),
           "choices": {}, "ms": {}}
    for M in sorted({int(m) for m in Ms}):
        n, xh = _batch(M, series, n_lo, n_hi, seed + M)
        x = torch.from_numpy(xh).to(device)
        best, timing = None, {}
        for tile in CANDIDATES[path]:
            plan = BatchPlan(n, [M] * len(n), path=path, tile=[tile] * len(n))
            bispectrum_batched_timed(x, plan)          # warm-up, allocation
            ts = [bispectrum_batched_timed(x, plan)[2]["contract"] for _ in range(reps)]
            timing[tile] = float(np.median(ts))
            if best is None or timing[tile] < timing[best]:
                best = tile
            del plan
        out["choices"][M] = best
        out["ms"][M] = timing
    if cache:
        d = os.path.dirname(os.path.abspath(cache))
        os.makedirs(d, exist_ok=True)
        with open(cache, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
    return out


def load(cache):
    """The choices of a saved tuning as {M: tile}."""
    with open(cache) as f:
        d = json.load(f)
    return {int(k): int(v) for k, v in d["choices"].items()}
