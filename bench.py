#!/usr/bin/env python3
"""Throughput of the bispectrum path on one MI355X.

Workload: one float32 series of n = 2^20 samples from the quadratic process
x_t = e_t + 0.5 e_{t-1} e_{t-2} (seeded), maximum lag M = 512, Parzen lag
window, 1024 x 1024 DFT.  A step is one full call of hos_bispectrum: mean
removal, operand preparation, the c3 contraction, the partial reduction,
mirroring + window and the 2D DFT, with the input already resident on the
GPU.  Metric: cumulant lag-sums per second, n (2M+1)^2 / step time.

Reported for the split-precision FP16 path (the headline ``value``), the
FP32 path and the split BF16 path, each with its normwise error against the
FP64 oracle on sampled lags; ``roofline`` is for the dominant kernel (the
contraction), timed with HIP events on the stream it runs on; the oracle is
timed on the host cores on a bounded sample of lags (``cpu_baseline``).

A second record inside the line, ``trispectrum``, measures the fourth-order
path on its own workload: n = 2^18 float32 samples of the cubic process
x_t = e_t + 0.4 e_{t-1} e_{t-2} e_{t-3}, M = 48, six-factor Parzen window,
96^3 DFT; metric n (2M+1)^3 lag-sums per second.  Further records:
``batched`` (4096 uneven series in one call), ``loss`` (bispectrum-matching
loss forward and adjoint), ``segments`` (the headline series in 16
segments, each centred on its own mean, cumulants averaged), ``order5``
(the fifth cumulant and its 4-D spectrum, n = 2^18, M = 24), ``streamed``
(a host-resident record of 2^26 samples read in pieces, host-to-device
copies inside the timed region) and
``direct_method`` (Algorithm DBS with
window-sum smoothing, n = 2^16 as one part, 1023 x 1023 box, with an HBM
roofline of the smoothing kernel).

``traffic`` (HBM bytes per launch of the contraction) is read from the
committed PMC summary when the contraction's source still matches the one it
was measured on, else null.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cumulant lag-sums/s (n·(2M+1)^2/s), split-prec vs FP32 at ≤1e-5 rel err"
METRIC4 = "cumulant lag-sums/s (n·(2M+1)^3/s)"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_c3_contract_n2p20_M512_traffic.txt")
MFMA_BUSY_FILE = os.path.join(ROOT, "profiles", "k_c3_contract_n2p20_M512_mfma_busy.txt")
C3_SOURCE = os.path.join(ROOT, "paper_1805_11775_amd", "csrc", "k_c3.hip")
DBS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dbs_box_n2p16_M3_1023_traffic.txt")
DBS_SOURCE = os.path.join(ROOT, "paper_1805_11775_amd", "csrc", "k_dbs.hip")
PEAK = {"fp32": 157.3e12, "split_fp16": 2.5166e15, "split_bf16": 2.5166e15}
DTYPE = {"fp32": "f32", "split_fp16": "f16", "split_bf16": "bf16"}
TOL = {"fp32": 1e-6, "split_fp16": 1e-5, "split_bf16": 1e-5}


def sample_lags(M, k, seed=11):
    rng = np.random.default_rng(seed)
    w1 = rng.integers(-M, M + 1, k)
    w2 = np.clip(w1 + rng.integers(-M, M + 1, k), -M, M)
    orbit = np.array([[1, 2], [2, 1], [-1, 1], [1, -1], [-2, -1], [-1, -2], [0, 0]])
    return np.concatenate([orbit[:, 0], w1]), np.concatenate([orbit[:, 1], w2])


def graph_replay_ms(torch, call, steps, warmup):
    """ms per replay of one call captured in a HIP graph: the same kernels on
    the same (resident) input, without the host's per-launch overhead.  The
    warm-up runs on a side stream of default priority, as capture wants; the
    call must enqueue on the current stream."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_path(hos, torch, xt, M, N, path, steps, warmup):
    n = xt.numel()
    pth = hos.PATHS[path]
    wsb = hos.hos_bispectrum_workspace(n, M, N, pth)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    c3 = torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64, device="cuda")
    B = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    stream = hos._stream_handle(xt.device)
    args = (xt.data_ptr(), hos.HOS_F32, n, M, hos.HOS_WIN_PARZEN, N, pth, 0,
            c3.data_ptr(), B.data_ptr(), ws.data_ptr(), wsb, stream)

    def call():
        st = hos.hos_bispectrum(*args)
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_bispectrum")

    def call_current():
        st = hos.hos_bispectrum(*args[:-1], hos._stream_handle(xt.device))
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_bispectrum")

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # per-stage durations: HIP events recorded by the library on `stream`
    stages = []
    for _ in range(5):
        st, d = hos.hos_bispectrum_timed(*args)
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_bispectrum_timed")
        stages.append(d)
    stage_ms = {k: float(np.mean([d[k] for d in stages])) for k in stages[0]}
    # the returned c3 is the last graph replay's: the error check covers it
    gms = graph_replay_ms(torch, call_current, steps, warmup)
    return ms, stage_ms, c3.cpu().numpy(), gms


def run_tri_path(hos, torch, xt, M, N, path, steps, warmup):
    n = xt.numel()
    pth = hos.PATHS[path]
    wsb = hos.hos_trispectrum_workspace(n, M, N, pth)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    c4 = torch.empty((2 * M + 1,) * 3, dtype=torch.float64, device="cuda")
    T = torch.empty((N, N, N), dtype=torch.complex128, device="cuda")
    stream = hos._stream_handle(xt.device)
    args = (xt.data_ptr(), hos.HOS_F32, n, M, hos.HOS_WIN_PARZEN, N, pth, 0,
            c4.data_ptr(), T.data_ptr(), ws.data_ptr(), wsb, stream)

    def call():
        st = hos.hos_trispectrum(*args)
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_trispectrum")

    def call_current():
        st = hos.hos_trispectrum(*args[:-1], hos._stream_handle(xt.device))
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_trispectrum")

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stages = []
    for _ in range(5):
        st, d = hos.hos_trispectrum_timed(*args)
        if st != hos.HOS_OK:
            raise hos.HosError(st, "hos_trispectrum_timed")
        stages.append(d)
    stage_ms = {k: float(np.mean([d[k] for d in stages])) for k in stages[0]}
    gms = graph_replay_ms(torch, call_current, steps, warmup)
    return ms, stage_ms, c4.cpu().numpy(), gms


def bench_trispectrum(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds):
    x, cfg = synth.workload_trispectrum()
    M, N = cfg["M"], cfg["nfft"]
    n = x.size
    xt = torch.from_numpy(x).cuda()
    lagsums = n * (2 * M + 1) ** 3
    flops = 2.0 * n * (M + 1) * (M + 2) * (M + 3) / 6  # one MAC per (i, a, b, c) of F4
    rng = np.random.default_rng(12)
    t = np.concatenate([[[1, 2, 3], [0, 0, 0], [3, 2, 1]], rng.integers(-M, M + 1, (200, 3))])
    ref = oracle.c4_at(x, t[:, 0], t[:, 1], t[:, 2])
    span = np.maximum(t.max(1), 0) - np.minimum(t.min(1), 0)
    ref[span > M] = 0.0
    m4_0 = float(oracle.m4_at(x, [0], [0], [0])[0])
    out = {}
    for path in paths:
        print("bench: trispectrum path %s" % path, file=sys.stderr, flush=True)
        ms, stage_ms, c4, gms = run_tri_path(hos, torch, xt, M, N, path, steps, warmup)
        got = c4[t[:, 0] + M, t[:, 1] + M, t[:, 2] + M]
        err = float(np.max(np.abs(got - ref)) / m4_0)
        t_k = stage_ms["contract"] * 1e-3
        out[path] = {"ms_per_step": ms, "value": lagsums / (ms * 1e-3), "rel_err_m4": err,
                     "graph_ms_per_step": gms,
                     "within_tol": err <= TOL[path], "stage_ms": stage_ms,
                     "contract_tflops": flops / t_k / 1e12,
                     "contract_frac": flops / t_k / PEAK[path]}
        print("bench: trispectrum %s %.3f ms/step, contract %.3f ms, err %.2e" %
              (path, ms, stage_ms["contract"], err), file=sys.stderr, flush=True)
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    hp = out[head]
    t_k = hp["stage_ms"]["contract"] * 1e-3
    rec = {"metric": METRIC4, "value": hp["value"], "unit": "lag-sums/s",
           "ms_per_step": hp["ms_per_step"], "dtype": DTYPE[head],
           "config": {"workload": "trispectrum of one n=2^18 float32 cubic-process series "
                                  "(x_t = e_t + 0.4 e_{t-1} e_{t-2} e_{t-3}), M=48, "
                                  "six-factor Parzen window, 96^3 DFT",
                      "n": n, "M": M, "nfft": N, "path": head},
           "roofline": {"bound": "mfma", "kernel": "k_c4_contract",
                        "achieved": flops / t_k / 1e12, "peak": PEAK[head] / 1e12,
                        "unit": "TFLOP/s", "frac": flops / t_k / PEAK[head], "traffic": None,
                        "flops_per_launch": flops, "avg_launch_ms": hp["stage_ms"]["contract"]},
           "paths": out}
    if cpu_seconds > 0:
        # the oracle's c4 at a bounded sample of lags of the same series
        t0 = time.perf_counter()
        k = 16
        while True:
            tt = rng.integers(-M, M + 1, (k, 3))
            oracle.c4_at(x, tt[:, 0], tt[:, 1], tt[:, 2])
            el = time.perf_counter() - t0
            if el > cpu_seconds or k > 1 << 22:
                break
            k *= 2
            t0 = time.perf_counter()
        rec["cpu_oracle"] = {"value": k * n / el, "unit": "lag-sums/s", "kind": "oracle",
                             "sample": "%d random lags x n=%d, FP64 brute-force c4 (%.1f s)"
                                       % (k, n, el)}
    return rec


def bench_cumulant5(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds):
    """Order five: n = 2^18 float32 quartic process, M = 24, ten-difference
    Parzen window, 48^4 DFT; metric n (2M+1)^4 lag-sums/s; roofline of the
    fifth-moment contraction (one MAC per (i, a, b, c, d) of F5)."""
    x, cfg = synth.workload_cumulant5()
    M, N = cfg["M"], cfg["nfft"]
    n = x.size
    xt = torch.from_numpy(x).cuda()
    lagsums = float(n) * (2 * M + 1) ** 4
    flops = 2.0 * n * (M + 1) * (M + 2) * (M + 3) * (M + 4) / 24
    rng = np.random.default_rng(14)
    t = np.concatenate([[[1, 2, 3, 4], [0, 0, 0, 0]], rng.integers(-M, M + 1, (120, 4))])
    ref = oracle.c5_at(x, t[:, 0], t[:, 1], t[:, 2], t[:, 3])
    span = np.maximum(t.max(1), 0) - np.minimum(t.min(1), 0)
    ref[span > M] = 0.0
    scale = float(np.mean(np.abs(x.astype(np.float64) - np.mean(x.astype(np.float64))) ** 5))
    out = {}
    ws = None
    for path in paths:
        print("bench: order five path %s" % path, file=sys.stderr, flush=True)
        c5, _ = hos.cumulant5(xt, M, N, path=path)
        ms = _time(torch, lambda: hos.cumulant5(xt, M, N, path=path), max(3, steps // 5),
                   max(2, warmup // 5))
        st = [hos.cumulant5(xt, M, N, path=path, timed=True)[2] for _ in range(5)]
        stage_ms = {k: float(np.median([d[k] for d in st])) for k in st[0]}
        got = c5.cpu().numpy()[t[:, 0] + M, t[:, 1] + M, t[:, 2] + M, t[:, 3] + M]
        err = float(np.max(np.abs(got - ref)) / scale)
        t_k = stage_ms["contract"] * 1e-3
        out[path] = {"ms_per_step": ms, "value": lagsums / (ms * 1e-3), "rel_err_m5abs": err,
                     "within_tol": err <= TOL[path], "stage_ms": stage_ms,
                     "contract_tflops": flops / t_k / 1e12,
                     "contract_frac": flops / t_k / PEAK[path]}
        print("bench: order five %s %.3f ms/step, contract %.3f ms, err %.2e" %
              (path, ms, stage_ms["contract"], err), file=sys.stderr, flush=True)
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    hp = out[head]
    t_k = hp["stage_ms"]["contract"] * 1e-3
    rec = {"metric": "cumulant lag-sums/s (n·(2M+1)^4/s)", "value": hp["value"],
           "unit": "lag-sums/s", "ms_per_step": hp["ms_per_step"], "dtype": DTYPE[head],
           "config": {"workload": "order-five cumulant and 4-D spectrum of one n=2^18 float32 "
                                  "quartic-process series (x_t = e_t + 0.3 e_{t-1} e_{t-2} "
                                  "e_{t-3} e_{t-4}), M=24, ten-difference Parzen window, "
                                  "48^4 DFT",
                      "n": n, "M": M, "nfft": N, "path": head},
           "roofline": {"bound": "mfma", "kernel": "k_c5_contract",
                        "achieved": flops / t_k / 1e12, "peak": PEAK[head] / 1e12,
                        "unit": "TFLOP/s", "frac": flops / t_k / PEAK[head], "traffic": None,
                        "flops_per_launch": flops, "avg_launch_ms": hp["stage_ms"]["contract"]},
           "paths": out}
    if cpu_seconds > 0:
        t0 = time.perf_counter()
        k = 16
        while True:
            tt = rng.integers(-M, M + 1, (k, 4))
            oracle.c5_at(x, tt[:, 0], tt[:, 1], tt[:, 2], tt[:, 3])
            el = time.perf_counter() - t0
            if el > cpu_seconds or k > 1 << 20:
                break
            k *= 2
            t0 = time.perf_counter()
        rec["cpu_oracle"] = {"value": k * n / el, "unit": "lag-sums/s", "kind": "oracle",
                             "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                         len(os.sched_getaffinity(0)))),
                             "sample": "%d random lags x n=%d, FP64 brute-force c5 (%.1f s)"
                                       % (k, n, el)}
    return rec


def _time(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds=0.0):
    """4096 float32 series of uneven length and lag in one batched call
    (principal-domain spectra only); metric sum_s n_s (2 M_s + 1)^2 / t."""
    xs, n, M = synth.workload_batched()
    x = torch.from_numpy(np.concatenate(xs).astype(np.float32)).cuda()
    lagsums = float(np.sum(n * (2 * M + 1.0) ** 2))
    flops = float(np.sum(2.0 * n * (M + 1.0) * (M + 2.0) / 2))
    from paper_1805_11775_amd import tune as hos_tune
    out = {}
    for path in paths:
        # the shipped table tuned on this device (the tests' plan too), else tune now
        table = hos_tune.load(hos_tune.device_key(path))
        source = "shipped table (%s)" % os.path.basename(hos_tune.SHIPPED)
        if table is None:
            print("bench: batched path %s (tuning tiles)" % path, file=sys.stderr, flush=True)
            table = hos_tune.tune(sorted(set(int(m) for m in M)), path=path, series=32, reps=3)
            source = "tuned in this run"
        print("bench: batched path %s, tiles from the %s" % (path, source), file=sys.stderr,
              flush=True)
        plan = hos.BatchPlan(n, M, path=path, tile=hos_tune.tiles_for(n, M, table))
        plan.to(x.device)
        ms = _time(torch, lambda: hos.bispectrum_batched(x, plan, return_c3=False),
                   max(2, steps // 10), max(1, warmup // 10))
        stages = [hos.bispectrum_batched_timed(x, plan)[2] for _ in range(3)]
        stage_ms = {k: float(np.mean([d[k] for d in stages])) for k in stages[0]}
        _, B = hos.bispectrum_batched(x, plan, return_c3=False)
        S = plan.series()
        s = int(np.argmin(n))
        N, npd, pdo = int(S[s, 2]), int(S[s, 3]), int(S[s, 6])
        _, Bref = oracle.bispectrum(xs[s].astype(np.float32), int(M[s]), N)
        k1, k2 = oracle.pd_indices(N)
        err = float(np.max(np.abs(B[pdo:pdo + npd].cpu().numpy() - Bref[k1, k2])) /
                    np.max(np.abs(Bref[k1, k2])))
        out[path] = {"ms_per_call": ms, "value": lagsums / (ms * 1e-3),
                     "tflops_whole_call": flops / (ms * 1e-3) / 1e12,
                     "stage_ms": stage_ms,
                     "contract_tflops": flops / (stage_ms["contract"] * 1e-3) / 1e12,
                     "contract_frac": flops / (stage_ms["contract"] * 1e-3) / PEAK[path],
                     "frac_whole_call": flops / (ms * 1e-3) / PEAK[path],
                     "rel_err_B_pd_shortest_series": err, "within_tol": err <= TOL[path],
                     "tile_choices": {str(k): v for k, v in table["choices"].items()},
                     "tile_buckets": table["edges"], "tile_source": source,
                     "work_items": [plan.info["items0"], plan.info["items1"]],
                     "workgroups": [plan.info["G0"], plan.info["G1"]],
                     "ws_bytes": plan.info["ws_bytes"]}
        print("bench: batched %s %.3f ms/call, err %.2e" % (path, ms, err), file=sys.stderr,
              flush=True)
        del plan
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    h = out[head]
    rec = {"metric": "cumulant lag-sums/s (sum_s n_s (2M_s+1)^2 / s)",
           "value": h["value"], "unit": "lag-sums/s",
           "ms_per_step": h["ms_per_call"], "dtype": DTYPE[head],
           "config": {"workload": "4096 float32 series, n uniform in [1024, 65536], M uniform "
                                  "in {32, 64, 128, 256}, even index N(0,1), odd index "
                                  "Exp(1)-1; Parzen window, N = 2M; principal-domain spectra; "
                                  "tiles from the autotuner (per lag and length bucket)",
                      "series": len(n), "samples": int(np.sum(n)), "path": head},
           # one persistent launch over the work items of both tile classes
           # (4 x 4 and 2 x 2 blocks; k_c3_items_u, or k_c3_items on the FP32 path)
           "roofline": {"bound": "mfma", "kernel": "k_c3_items_u" if head != "fp32" else "k_c3_items",
                        "achieved": h["contract_tflops"], "peak": PEAK[head] / 1e12,
                        "unit": "TFLOP/s", "frac": h["contract_frac"], "traffic": None,
                        "flops_per_call": flops, "avg_call_ms": h["stage_ms"]["contract"]},
           "paths": out}
    if cpu_seconds > 0:
        t0 = time.perf_counter()
        k = lagsums_done = 0
        w1, w2 = sample_lags(64, 64, seed=19)
        while time.perf_counter() - t0 < cpu_seconds:
            s_ = (37 * k) % len(n)
            m = int(M[s_])
            sel = (np.abs(w1) <= m) & (np.abs(w2) <= m) & (np.abs(w1 - w2) <= m)
            oracle.c3_at(xs[s_], w1[sel], w2[sel])
            lagsums_done += int(sel.sum()) * xs[s_].size
            k += 1
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"value": lagsums_done / t, "unit": "lag-sums/s",
                             "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                         len(os.sched_getaffinity(0)))),
                             "kind": "oracle",
                             "sample": "%d series of the batch x up to 64 lags |w| <= 64, "
                                       "FP64 brute-force c3 (%.1f s)" % (k, t)}
    return rec


def bench_loss(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds=0.0):
    """Loss forward and hand-written backward over 64 float32 N(0,1) series,
    n = 65536, M = 256, N = 512."""
    X, tgt, cfg = synth.workload_loss()
    M, N = cfg["M"], cfg["nfft"]
    B_, n_ = X.shape
    x = torch.from_numpy(X).cuda()
    _, target = hos.bispectrum_batched(torch.from_numpy(tgt.astype(np.float32)).cuda(),
                                       hos.BatchPlan([tgt.size], [M], path="fp32"),
                                       return_c3=False)
    lagsums = float(B_ * n_ * (2 * M + 1) ** 2)
    hexagon = 3 * M * M + 3 * M + 1
    fwd_flops = B_ * 2.0 * n_ * (M + 1) * (M + 2) / 2
    # the quadratic form of the (2M+1)-sample window over the hexagon has a
    # symmetric kernel: one MAC per unordered lag pair, (|H| + 2M + 1) / 2
    bwd_flops = B_ * float(n_) * (hexagon + 2 * M + 1)
    # the smallest count of the adjoint: the lag weights folded onto F and the
    # two products Z = H G_F^T, Z' = H G_F (one MAC per sample and F entry
    # each), 2 n (M+1)(M+2) FLOP per series
    bwd_flops_fold = B_ * 2.0 * n_ * (M + 1) * (M + 2)
    dL = torch.ones((), dtype=torch.float64, device="cuda")
    out = {}
    for path in paths:
        print("bench: loss path %s" % path, file=sys.stderr, flush=True)
        plan = hos.BatchPlan([n_] * B_, [M] * B_, path=path, adjoint=True)
        plan.to(x.device)
        loss, Bpd = hos.bispectrum_loss_fwd(x, target, plan)
        t_f = _time(torch, lambda: hos.bispectrum_loss_fwd(x, target, plan),
                    max(2, steps // 5), max(1, warmup // 5))
        t_b = _time(torch, lambda: hos.bispectrum_loss_bwd(x, target, Bpd, dL, plan),
                    max(2, steps // 5), max(1, warmup // 5))
        b = 37
        Bref = oracle.bispectrum_pd(X[b], M, N)
        npd = Bpd.numel() // B_
        err = float(np.max(np.abs(Bpd[b * npd:(b + 1) * npd].cpu().numpy() - Bref)) /
                    np.max(np.abs(Bref)))
        out[path] = {"fwd_ms": t_f, "bwd_ms": t_b, "fwd_value": lagsums / (t_f * 1e-3),
                     "fwd_tflops": fwd_flops / (t_f * 1e-3) / 1e12,
                     "bwd_tflops": bwd_flops / (t_b * 1e-3) / 1e12,
                     "bwd_frac": bwd_flops / (t_b * 1e-3) / PEAK[path],
                     "bwd_frac_fold_count": bwd_flops_fold / (t_b * 1e-3) / PEAK[path],
                     "loss": float(loss), "rel_err_B_pd_series37": err,
                     "within_tol": err <= TOL[path]}
        print("bench: loss %s fwd %.3f ms bwd %.3f ms err %.2e" % (path, t_f, t_b, err),
              file=sys.stderr, flush=True)
        del plan
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    h = out[head]
    rec = {"metric": "forward lag-sums/s; backward ms", "value": h["fwd_value"],
           "unit": "lag-sums/s", "dtype": DTYPE[head],
           "config": {"workload": "bispectrum-matching loss, 64 float32 N(0,1) series, "
                                  "n=65536, M=256, N=512, target from a quadratic-process "
                                  "series; forward + hand-written adjoint",
                      "batch": B_, "n": n_, "M": M, "nfft": N, "path": head},
           "bwd_flops_definition": "n (|H| + 2M + 1) per series, |H| = 3M^2+3M+1: one MAC "
                                   "per unordered lag pair of the symmetric quadratic form of "
                                   "the (2M+1)-sample window over the hexagon; "
                                   "bwd_frac_fold_count prices the call at the folded "
                                   "count 2 n (M+1)(M+2) per series instead",
           "bwd_flops_fold": bwd_flops_fold,
           # the backward entry point has no stage events: the whole backward
           # call is timed, so the adjoint contraction's own fraction (see its
           # kernel trace) is higher than this one
           "roofline": {"bound": "mfma", "kernel": "k_adj_contract",
                        "achieved": h["bwd_tflops"], "peak": PEAK[head] / 1e12,
                        "unit": "TFLOP/s", "frac": h["bwd_frac"], "traffic": None,
                        "flops_per_call": bwd_flops, "avg_call_ms": h["bwd_ms"],
                        "timed": "whole backward call"},
           "paths": out}
    if cpu_seconds > 0:
        t0 = time.perf_counter()
        oracle.bispectrum_pd(X[0], M, N)
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"value": n_ * (2 * M + 1) ** 2 / t, "unit": "lag-sums/s",
                             "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                         len(os.sched_getaffinity(0)))),
                             "kind": "oracle",
                             "sample": "the forward of one series of the 64 (c3 over the "
                                       "hexagon by FP64 brute force, window, DFT; %.1f s)" % t}
    return rec


def bench_segments(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds):
    """Segment averaging: the headline series cut into 16 segments of
    65536 samples, each centred on its own mean, c3 averaged, Parzen window,
    1024 x 1024 DFT; metric n (2M+1)^2 lag-sums/s as for one series.  The
    contraction (k_c3_items over the 16 segments) is timed by the batched
    entry point's stage events on the same plan."""
    x, cfg = synth.workload_segments()
    P, M = cfg["P"], cfg["M"]
    K = x.size // P
    xt = torch.from_numpy(x).cuda()
    lagsums = float(K * P) * (2 * M + 1) ** 2
    flops = K * 2.0 * P * (M + 1) * (M + 2) / 2
    w1, w2 = sample_lags(M, 120, seed=13)
    ref = np.mean([oracle.c3_at(x[i * P:(i + 1) * P], w1, w2) for i in range(K)], 0)
    ref[np.abs(w1 - w2) > M] = 0.0
    out = {}
    for path in paths:
        plan = hos.BatchPlan([P] * K, [M] * K, path=path, segments=True)
        ms = _time(torch, lambda: hos.bispectrum_segments(xt, P, M, path=path, plan=plan),
                   max(3, steps // 5), max(2, warmup // 5))
        st = [hos.bispectrum_batched_timed(xt, plan)[2] for _ in range(3)]
        stage_ms = {k: float(np.median([d[k] for d in st])) for k in st[0]}
        c3, _ = hos.bispectrum_segments(xt, P, M, path=path, plan=plan)
        c3 = c3.cpu().numpy()
        err = float(np.max(np.abs(c3[w1 + M, w2 + M] - ref)) / np.max(np.abs(ref)))
        out[path] = {"ms_per_call": ms, "value": lagsums / (ms * 1e-3), "rel_err": err,
                     "within_tol": err <= TOL[path], "batched_stage_ms": stage_ms,
                     "contract_tflops": flops / (stage_ms["contract"] * 1e-3) / 1e12,
                     "contract_frac": flops / (stage_ms["contract"] * 1e-3) / PEAK[path]}
        print("bench: segments %s %.3f ms/call, err %.2e" % (path, ms, err), file=sys.stderr,
              flush=True)
        del plan
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    h = out[head]
    rec = {"metric": METRIC, "value": h["value"], "unit": "lag-sums/s",
           "ms_per_step": h["ms_per_call"], "dtype": DTYPE[head],
           "config": {"workload": "segment-averaged bispectrum: n=2^20 float32 quadratic "
                                  "process in 16 segments of 65536 (each centred on its own "
                                  "mean), M=512, Parzen window, 1024x1024 DFT",
                      "n": int(K * P), "P": P, "K": K, "M": M, "path": head},
           "roofline": {"bound": "mfma", "kernel": "k_c3_items",
                        "achieved": flops / (h["batched_stage_ms"]["contract"] * 1e-3) / 1e12,
                        "peak": PEAK[head] / 1e12, "unit": "TFLOP/s",
                        "frac": h["contract_frac"], "traffic": None,
                        "flops_per_launch": flops,
                        "avg_launch_ms": h["batched_stage_ms"]["contract"]},
           "paths": out}
    if cpu_seconds > 0:
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < cpu_seconds:
            oracle.c3_at(x[k % K * P:(k % K + 1) * P], w1, w2)
            k += 1
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"value": k * w1.size * P / t, "unit": "lag-sums/s",
                             "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                         len(os.sched_getaffinity(0)))),
                             "kind": "oracle",
                             "sample": "%d segments x %d lags x %d samples, FP64 brute-force "
                                       "c3 (%.1f s)" % (k, w1.size, P, t)}
    return rec


def bench_streamed(hos, torch, oracle, synth, paths, steps, warmup, cpu_seconds):
    """A record in pinned host memory streamed through the device
    (hos_bispectrum_streamed): n = 2^26 float32 quadratic process, M = 512,
    Parzen window, 1024 x 1024 DFT, pieces of 2^22 samples.  The time runs
    from the host-resident record to c3 and B on the device, so it includes
    both passes of host-to-device copies; beside it, the in-memory call on
    the same record already resident in HBM and a plain copy of the record
    to the device (the host link's rate)."""
    x, cfg = synth.workload_streamed()
    M, N, piece = cfg["M"], cfg["nfft"], cfg["piece"]
    n = x.size
    xh = torch.from_numpy(x).pin_memory()
    xd = torch.empty(n, dtype=torch.float32, device="cuda")
    copy_ms = _time(torch, lambda: xd.copy_(xh, non_blocking=True), 5, 2)
    lagsums = float(n) * (2 * M + 1) ** 2
    flops = 2.0 * n * (M + 1) * (M + 2) / 2
    w1, w2 = sample_lags(M, 40, seed=17)
    ref = oracle.c3_at(x, w1, w2)
    ref[np.abs(w1 - w2) > M] = 0.0
    reps, warm = max(3, steps // 10), max(1, warmup // 10)
    out = {}
    for path in paths:
        wsb = hos.hos_bispectrum_workspace(n, M, N, hos.PATHS[path], 0)
        wsm = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        mem_ms = _time(torch, lambda: hos.bispectrum(xd, M, N, path=path, workspace=wsm),
                       reps, warm)
        cm, _ = hos.bispectrum(xd, M, N, path=path, workspace=wsm)
        cm = cm.cpu().numpy()
        del wsm
        c3, _ = hos.bispectrum_streamed(xh, M, piece=piece, nfft=N, path=path)
        sz = hos.hos_bispectrum_streamed_workspace(n, M, N, hos.PATHS[path], hos.HOS_F32,
                                                   piece)
        wss = torch.empty(sz, dtype=torch.uint8, device="cuda")
        ms = _time(torch, lambda: hos.bispectrum_streamed(xh, M, piece=piece, nfft=N, path=path,
                                                         workspace=wss), reps, warm)
        c3 = c3.cpu().numpy()
        err = float(np.max(np.abs(c3[w1 + M, w2 + M] - ref)) / np.max(np.abs(ref)))
        dmem = float(np.max(np.abs(c3 - cm)) / np.max(np.abs(cm)))
        out[path] = {"ms_per_call": ms, "value": lagsums / (ms * 1e-3), "rel_err": err,
                     "within_tol": err <= TOL[path], "in_memory_ms": mem_ms,
                     "rel_diff_vs_in_memory": dmem, "workspace_bytes": sz,
                     "in_memory_workspace_bytes": wsb,
                     "pass2_copy_hidden_frac": (mem_ms + 2 * copy_ms - ms) / copy_ms}
        print("bench: streamed %s %.2f ms/call (in memory %.2f, copy %.2f), err %.2e" %
              (path, ms, mem_ms, copy_ms, err), file=sys.stderr, flush=True)
        del wss
    head = "split_fp16" if "split_fp16" in out else next(iter(out))
    h = out[head]
    link_bytes = 2.0 * n * 4 + (n // piece) * M * 4   # both passes, with the halos
    rec = {"metric": METRIC, "value": h["value"], "unit": "lag-sums/s",
           "ms_per_step": h["ms_per_call"], "dtype": DTYPE[head],
           "config": {"workload": "streamed bispectrum of a host-resident n=2^26 float32 "
                                  "quadratic-process record (pinned), M=512, Parzen window, "
                                  "1024x1024 DFT, pieces of 2^22 samples",
                      "n": n, "M": M, "nfft": N, "piece": piece, "path": head},
           "host_link": {"bytes_per_call": link_bytes,
                         "achieved_GBps": link_bytes / (h["ms_per_call"] * 1e-3) / 1e9,
                         "plain_copy_GBps": n * 4 / (copy_ms * 1e-3) / 1e9,
                         "plain_copy_ms": copy_ms},
           # pass one (the record's mean and scale) must end before any
           # operand is formed, so it cannot overlap compute: the two-pass
           # bound is the in-memory call plus one copy of the record
           "bound_ms": {"in_memory": h["in_memory_ms"], "one_copy": copy_ms,
                        "two_pass": h["in_memory_ms"] + copy_ms,
                        "frac": (h["in_memory_ms"] + copy_ms) / h["ms_per_call"]},
           "paths": out}
    del xd
    if cpu_seconds > 0:
        # the oracle runs its lags in parallel: 16 lags of the sample per call
        x64 = x.astype(np.float64)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < cpu_seconds:
            j = (16 * k) % (w1.size - 15)
            oracle.c3_at(x64, w1[j:j + 16], w2[j:j + 16])
            k += 1
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"value": 16 * k * float(n) / t, "unit": "lag-sums/s",
                             "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                         len(os.sched_getaffinity(0)))),
                             "kind": "oracle",
                             "sample": "%d lags x %d samples, FP64 brute-force c3 (%.1f s)" %
                                       (16 * k, n, t)}
    return rec


def bench_dbs(hos, torch, oracle, synth, steps, warmup, cpu_seconds, sweep_box=True):
    """The direct method (Algorithm DBS with window-sum smoothing): one
    float32 quadratic-process series of 2^16 samples as one part, a
    1023 x 1023 box; metric smoothed principal-domain points per second.
    Roofline of the smoothing kernel against HBM: its algorithmic traffic is
    the principal-domain output (16 B a point; the 1 MB spectrum it reads is
    L2-resident)."""
    x, cfg = synth.workload_dbs()
    P, M3 = cfg["P"], cfg["M3"]
    xt = torch.from_numpy(x).cuda()
    info = hos.hos_dbs_plan_info(x.size, P, M3)
    ws = torch.empty(info["ws_bytes"], dtype=torch.uint8, device="cuda")
    npd = info["npd"]
    print("bench: direct method n=%d M3=%d" % (x.size, M3), file=sys.stderr, flush=True)
    ms = _time(torch, lambda: hos.dbs(xt, P, M3, workspace=ws), max(3, steps // 5),
               max(2, warmup // 5))
    stages = [hos.dbs(xt, P, M3, workspace=ws, timed=True)[1] for _ in range(5)]
    stage_ms = {k: float(np.median([d[k] for d in stages])) for k in stages[0]}
    B = hos.dbs(xt, P, M3, workspace=ws).cpu().numpy()
    H = (P - 1) // 2
    rows = np.arange(H + 1)
    lens = np.minimum(rows, H - rows) + 1
    k1 = np.repeat(rows, lens)
    k2 = np.arange(k1.size) - np.repeat(np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    pick = np.random.default_rng(5).integers(0, npd, 12)
    ref = oracle.dbs_at(x, P, M3, k1[pick], k2[pick])
    err = float(np.max(np.abs(B[pick] - ref)) / np.max(np.abs(ref)))
    out_bytes = 16.0 * npd
    t_s = stage_ms["smooth"] * 1e-3
    sweep = {}
    for m3 in (5, 255) if sweep_box else ():
        st = [hos.dbs(xt, P, m3, workspace=None, timed=True)[1]["smooth"] for _ in range(4)]
        sweep[str(m3)] = {"smooth_ms": float(np.median(st)),
                          "hbm_frac": out_bytes / (np.median(st) * 1e-3) / 8.0e12}
    rec = {"metric": "smoothed bispectrum points/s (principal domain of the P grid)",
           "value": npd / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "dtype": "f64",
           "config": {"workload": "direct method (Algorithm DBS): one float32 "
                                  "quadratic-process series, n = 2^16, one part P = 2^16, "
                                  "box M3 = 1023, principal-domain output",
                      "n": int(x.size), "P": P, "M3": M3, "K": info["K"], "points": npd},
           "stage_ms": stage_ms, "rel_err_sampled": err, "within_tol": err <= 1e-10,
           "roofline": {"bound": "hbm", "kernel": "k_dbs_box",
                        "achieved": out_bytes / t_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": out_bytes / t_s / 8.0e12,
                        "traffic": traffic_record(DBS_TRAFFIC_FILE, DBS_SOURCE),
                        "bytes_per_launch": out_bytes, "avg_launch_ms": stage_ms["smooth"]},
           "box_sweep_same_series": sweep}
    if cpu_seconds > 0:
        # the oracle's explicit box sums at sampled points (M3^2 products each)
        t0 = time.perf_counter()
        oracle.dbs_at(x, P, M3, k1[:2], k2[:2])
        per = (time.perf_counter() - t0) / 2
        k = int(max(4, min(2000, cpu_seconds / max(per, 1e-9))))
        sel = np.random.default_rng(6).integers(0, npd, k)
        t0 = time.perf_counter()
        oracle.dbs_at(x, P, M3, k1[sel], k2[sel])
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"value": k / t, "unit": "points/s", "cores": 1, "kind": "oracle",
                             "sample": "%d principal-domain points, explicit %d x %d box "
                                       "sums in FP64 numpy (%.1f s)" % (k, M3, M3, t)}
    print("bench: direct method %.3f ms/call (smooth %.3f ms), err %.2e" %
          (ms, stage_ms["smooth"], err), file=sys.stderr, flush=True)
    return rec


def profile_value(path, key, source):
    """One figure of a committed PMC summary, if it was taken on the
    current kernel source; else None."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != hashlib.sha256(open(source, "rb").read()).hexdigest():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def traffic_record(path=TRAFFIC_FILE, source=C3_SOURCE):
    """HBM bytes per launch of a kernel from its committed PMC summary, if
    that was taken on the current kernel source."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = hashlib.sha256(open(source, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != src:
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def issued_flops(flops):
    """FLOP the split-FP16 c3 contraction issues per launch: its MFMA count
    from the committed PMC summary (while it matches the source) x 2*32*32*16,
    else three products per algorithmic MAC (which leaves out the blocks'
    triangle waste)."""
    n = profile_value(MFMA_BUSY_FILE, "sq_insts_mfma", C3_SOURCE)
    return n * 2.0 * 32 * 32 * 16 if n else 3.0 * flops


def ceiling_record(hos, path, issued_flops_per_s):
    """The measured matrix-core ceiling for ``path`` and the issued rate's
    fraction of it."""
    r = hos.mfma_rate(path, 1 << 19)
    return {"tflops": r["tflops"], "frac_of_peak": r["tflops"] * 1e12 / PEAK[path],
            "issued_tflops": issued_flops_per_s / 1e12,
            "issued_frac_of_ceiling": issued_flops_per_s / (r["tflops"] * 1e12),
            "probe": "4 waves/CU, 4 independent 32x32 MFMA chains, %.1f ms" % r["ms"]}


def cpu_baseline(oracle, x, M, seconds):
    """Oracle c3 (FP64 brute force, OpenMP) on a bounded sample of lags of
    the same series; rate in lag-sums/s."""
    n = x.size
    t0 = time.perf_counter()
    w1, w2 = sample_lags(M, 32, seed=3)
    oracle.c3_at(x, w1, w2)
    t_probe = time.perf_counter() - t0
    per_lag = t_probe / w1.size
    k = int(max(32, min(200000, seconds / max(per_lag, 1e-9))))
    w1, w2 = sample_lags(M, k, seed=4)
    t0 = time.perf_counter()
    oracle.c3_at(x, w1, w2)
    t = time.perf_counter() - t0
    return {"value": w1.size * n / t, "unit": "lag-sums/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "%d lags of the hexagon x n=%d samples, FP64 brute-force c3 "
                      "(%.1f s)" % (w1.size, n, t)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--paths", default="split_fp16,fp32,split_bf16")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tri", action="store_true", help="skip the trispectrum record")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and loss records")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streamed (host-resident record) record")
    ap.add_argument("--no-dbs", action="store_true", help="skip the direct-method record")
    ap.add_argument("--no-dbs-sweep", action="store_true",
                    help="time the direct method at its workload's box size only")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (the "
                         "reference kernel for scaling HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only (--gpus 1): the library has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    if "OMP_NUM_THREADS" not in os.environ:
        os.environ["OMP_NUM_THREADS"] = str(len(os.sched_getaffinity(0)))

    import torch

    import oracle
    import paper_1805_11775_amd as hos
    import synth

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy of %d bytes done" % nb, file=sys.stderr, flush=True)
        del src, dst

    x, cfg = synth.workload_long_bispectrum()
    M, N = cfg["M"], cfg["nfft"]
    n = x.size
    xt = torch.from_numpy(x).cuda()
    lagsums = n * (2 * M + 1) ** 2
    flops = 2.0 * n * (M + 1) * (M + 2) / 2  # one MAC per (i, a, b) of F

    w1, w2 = sample_lags(M, 200)
    ref = oracle.c3_at(x, w1, w2)
    ref[np.abs(w1 - w2) > M] = 0.0

    paths = {}
    for path in args.paths.split(","):
        print("bench: path %s" % path, file=sys.stderr, flush=True)
        ms, stage_ms, c3, gms = run_path(hos, torch, xt, M, N, path, args.steps, args.warmup)
        err = float(np.max(np.abs(c3[w1 + M, w2 + M] - ref)) / np.max(np.abs(ref)))
        t_k = stage_ms["contract"] * 1e-3
        paths[path] = {
            "ms_per_step": ms, "value": lagsums / (ms * 1e-3), "rel_err": err,
            "graph_ms_per_step": gms, "graph_value": lagsums / (gms * 1e-3),
            "within_tol": err <= TOL[path], "stage_ms": stage_ms,
            "contract_tflops": flops / t_k / 1e12,
            "contract_frac": flops / t_k / PEAK[path],
            "issued_mfma_frac": (3 if path != "fp32" else 1) * flops / t_k / PEAK[path],
        }
        print("bench: %s %.3f ms/step, contract %.3f ms, err %.2e" %
              (path, ms, stage_ms["contract"], err), file=sys.stderr, flush=True)

    head = "split_fp16" if "split_fp16" in paths else next(iter(paths))
    hp = paths[head]
    t_k = hp["stage_ms"]["contract"] * 1e-3
    rec = {
        "metric": METRIC, "value": hp["value"], "unit": "lag-sums/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hp["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head], "data": "synthetic",
        "config": {"workload": "bispectrum of one n=2^20 float32 quadratic-process series "
                               "(x_t = e_t + 0.5 e_{t-1} e_{t-2}), M=512, Parzen window, "
                               "1024x1024 DFT",
                   "n": n, "M": M, "nfft": N, "path": head},
        "roofline": {"bound": "mfma", "kernel": "k_c3_contract", "achieved": flops / t_k / 1e12,
                     "peak": PEAK[head] / 1e12, "unit": "TFLOP/s",
                     "frac": flops / t_k / PEAK[head], "traffic": traffic_record(),
                     "flops_per_launch": flops, "avg_launch_ms": hp["stage_ms"]["contract"],
                     # matrix-core busy cycles over the kernel's cycles (rocprofv3 PMC),
                     # issued work: three FP16 products per algorithmic MAC plus the
                     # blocks' triangle waste
                     "mfma_busy": profile_value(MFMA_BUSY_FILE, "mfma_busy_frac", C3_SOURCE),
                     # the matrix cores' attainable rate on this device, measured
                     # now (hos_mfma_rate: independent ops only), and the
                     # contraction's issued MFMA rate against it
                     "mfma_ceiling": ceiling_record(hos, head, issued_flops(flops) / t_k)},
        "paths": paths,
    }
    if not args.no_batch:
        rec["batched"] = bench_batched(hos, torch, oracle, synth, list(paths), args.steps,
                                       args.warmup, 0.0 if args.no_cpu_baseline else 3.0)
        rec["loss"] = bench_loss(hos, torch, oracle, synth, list(paths), args.steps,
                                 args.warmup, 0.0 if args.no_cpu_baseline else 1.0)
    if not args.no_tri:
        rec["trispectrum"] = bench_trispectrum(
            hos, torch, oracle, synth, list(paths), args.steps, args.warmup,
            0.0 if args.no_cpu_baseline else 5.0)
    if not args.no_tri:
        rec["order5"] = bench_cumulant5(hos, torch, oracle, synth, list(paths), args.steps,
                                        args.warmup, 0.0 if args.no_cpu_baseline else 3.0)
    if not args.no_batch:
        rec["segments"] = bench_segments(hos, torch, oracle, synth, list(paths), args.steps,
                                         args.warmup, 0.0 if args.no_cpu_baseline else 3.0)
    if not args.no_stream:
        rec["streamed"] = bench_streamed(hos, torch, oracle, synth, list(paths), args.steps,
                                         args.warmup, 0.0 if args.no_cpu_baseline else 3.0)
    if not args.no_dbs:
        rec["direct_method"] = bench_dbs(hos, torch, oracle, synth, args.steps, args.warmup,
                                         0.0 if args.no_cpu_baseline else 5.0,
                                         not args.no_dbs_sweep)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(oracle, x, M, args.cpu_seconds)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
