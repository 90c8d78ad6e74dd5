"""Tile tuner for the batched contraction, and its cache.

For every maximum lag M of a batch the contraction can run on tiles of
2 x 2 or 4 x 4 matrix-core blocks (split paths; the FP32 path has 4 x 4
tiles only).  Small tiles waste less of the triangle at small M, large tiles
reuse each product row across more columns.  The choice can also depend on
the series length (short series have few chunks per tile, so the tile count
and the per-item overheads weigh more).  ``tune`` asks the library's
``hos_tune`` to time both on the device for every (M, length bucket) -- a
synthetic batch per bucket, the contraction launch alone, the median of
several calls -- and keeps the faster.

The result is a table {(M, bucket): tile} stored as JSON under a key made of
the GPU architecture, its compute-unit count and the path, so one cache file
serves several machines and paths.  ``tiles_for(n, M, table)`` maps every
series of a batch to its (M, bucket) entry, for ``BatchPlan(..., tile=...)``.
The package ships the table tuned on MI355X for the benchmark's lags and
length range (``tuned_gfx950.json``).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import HOS_OK, PATHS, HosError, lib, _stream_handle

# length buckets of the benchmark's range [1024, 65536]: quarter-range steps
DEFAULT_EDGES = (1024, 4096, 16384, 32768, 65537)
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def device_key(path: str, device="cuda") -> str:
    """Cache key: architecture, compute units, path (e.g. 'gfx950:256:split_fp16')."""
    import torch
    p = torch.cuda.get_device_properties(torch.device(device))
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s:%d:%s" % (arch, p.multi_processor_count, path)


def tune(Ms, path="split_fp16", edges=DEFAULT_EDGES, series=32, reps=5, device="cuda",
         cache=None):
    """Times the tile candidates of every (M, length bucket) with hos_tune.

    Returns {"key": ..., "edges": [...], "choices": {M: [tile per bucket]},
    "ms": {M: [[ms tile 2, ms tile 4] per bucket]}}; with ``cache`` the entry
    is merged into that JSON file under its key."""
    import torch
    Ms = sorted({int(m) for m in Ms})
    edges = [int(e) for e in edges]
    nM, nb = len(Ms), len(edges) - 1
    Mc = (ctypes.c_int32 * nM)(*Ms)
    Ec = (ctypes.c_int64 * (nb + 1))(*edges)
    pth = PATHS[path]
    need = ctypes.c_size_t(0)
    st = lib().hos_tune_workspace(pth, Mc, nM, Ec, nb, int(series), ctypes.byref(need))
    if st != HOS_OK:
        raise HosError(st, "hos_tune_workspace")
    dev = torch.device(device)
    ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    tiles = (ctypes.c_int32 * (nM * nb))()
    ms = (ctypes.c_float * (nM * nb * 2))()
    st = lib().hos_tune(pth, Mc, nM, Ec, nb, int(series), int(reps), ctypes.c_void_p(ws.data_ptr()),
                        need.value, tiles, ms, _stream_handle(dev))
    if st != HOS_OK:
        raise HosError(st, "hos_tune")
    del ws
    out = {"key": device_key(path, device), "edges": edges, "series": int(series),
           "measure": "contraction launch, median ms of %d calls" % int(reps),
           "choices": {}, "ms": {}}
    for i, M in enumerate(Ms):
        out["choices"][M] = [int(tiles[i * nb + j]) for j in range(nb)]
        out["ms"][M] = [[round(float(ms[(i * nb + j) * 2 + c]), 5) for c in (0, 1)]
                        for j in range(nb)]
    if cache:
        save(out, cache)
    return out


def save(table, cache):
    """Merge one tuning result into the JSON cache file under its key."""
    data = {}
    if os.path.exists(cache):
        with open(cache) as f:
            data = json.load(f)
    data[table["key"]] = {"edges": table["edges"], "series": table["series"],
                          "measure": table["measure"],
                          "choices": {str(k): v for k, v in table["choices"].items()},
                          "ms": {str(k): v for k, v in table["ms"].items()}}
    d = os.path.dirname(os.path.abspath(cache))
    os.makedirs(d, exist_ok=True)
    with open(cache, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(key, cache=SHIPPED):
    """The cached table for ``key`` as {"edges": [...], "choices": {M: [tiles]}},
    or None when the cache has no such entry."""
    if not os.path.exists(cache):
        return None
    with open(cache) as f:
        data = json.load(f)
    e = data.get(key)
    if e is None:
        return None
    return {"edges": [int(v) for v in e["edges"]],
            "choices": {int(k): [int(t) for t in v] for k, v in e["choices"].items()}}


def tiles_for(n, M, table):
    """Per-series tile choices for a batch from a tuned table: series s takes
    the entry of its lag and of the bucket holding its length (0 -- the
    library's own rule -- for a lag the table does not cover)."""
    edges = np.asarray(table["edges"])
    out = []
    for ns, ms in zip(np.asarray(n).tolist(), np.asarray(M).tolist()):
        row = table["choices"].get(int(ms))
        if row is None:
            out.append(0)
            continue
        j = int(np.searchsorted(edges, ns, side="right")) - 1
        out.append(int(row[min(max(j, 0), len(row) - 1)]))
    return out


def main(argv=None):
    """``python -m paper_1805_11775_amd.tune --out FILE``: tune the batch
    workload's lags (32, 64, 128, 256) over its length range on every path
    and merge the tables into FILE (the shipped table was made this way)."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=SHIPPED)
    ap.add_argument("--lags", default="32,64,128,256")
    ap.add_argument("--paths", default="split_fp16,split_bf16,fp32")
    ap.add_argument("--series", type=int, default=32)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    for path in a.paths.split(","):
        t = tune([int(m) for m in a.lags.split(",")], path=path, series=a.series, reps=a.reps,
                 cache=a.out)
        print(t["key"], t["choices"], flush=True)


if __name__ == "__main__":
    main()
