#!/usr/bin/env python3
"""Localization throughput of the hloc hot path on one MI355X.

One step = one batch of query frames through the whole path: query prep,
coarse screen and FP64 region re-score, region scheduling, fine MFMA screen,
selection, FP64 rerank, and per-request aggregation, with inputs resident in
device memory. The default workload is the plain-FP32 shape: N = 200,000 rows
of D = 256, 1,024 regions of uneven size, 256 single-frame queries per batch,
8 regions per frame, k = 16.

Prints one JSON line: throughput (frames/s), per-step p50/p99, the roofline of
the fine screen (algorithmic bytes over its event-timed duration against HBM
peak), and the FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "localization queries/sec at recall@k=1.0 vs FP64 oracle; HBM GB/s % peak; p99 ms"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, gpu_idx, seconds: float):
    """Time the FP64 oracle on the first frames of the batch (about `seconds`
    of single-threaded work) and check the GPU's lists on them."""
    import oracle
    m = 4
    while True:
        t0 = time.perf_counter()
        ora = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, w.q[:m], w.k, w.n_reg)
        for r in range(m):
            oracle.aggregate(ora["idx"][r], w.xy, *w.agg)
        dt = time.perf_counter() - t0
        if dt >= seconds or m >= len(w.q):
            break
        m = min(len(w.q), max(m + 1, int(m * seconds / max(dt, 1e-3) * 1.1)))
    hits = sum(len(set(gpu_idx[i].tolist()) & set(ora["idx"][i].tolist())) for i in range(m))
    exact = sum(int(np.array_equal(gpu_idx[i], ora["idx"][i])) for i in range(m))
    return dict(value=m / dt, unit="queries/s", cores=1, kind="oracle",
                sample=f"first {m} of {len(w.q)} frames of {w.name}, single thread, "
                       f"{dt:.1f} s"), hits / (m * w.k), exact, m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", type=int, default=1, help="index of workload.SHAPES")
    ap.add_argument("--nq", type=int, default=None, help="override the batch size")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_08861_amd import hloc, workload

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = workload.make_workload(a.workload, nq=a.nq)
    log(f"[bench] workload {w.name}: n={len(w.feats)} d={w.feats.shape[1]} "
        f"regions={w.n_regions_total} frames={len(w.q)} requests={len(w.req_offsets) - 1} "
        f"({time.perf_counter() - t0:.1f} s)")
    db = hloc.HlocDB(w.feats, w.xy)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    nq, k, nreq = len(w.q), w.k, len(w.req_offsets) - 1
    db.reserve(nq, nreq, k, w.n_reg)
    q = torch.from_numpy(w.q).to(dev)
    offs = torch.from_numpy(w.req_offsets.astype(np.int32)).to(dev)
    idx = torch.empty((nq, k), dtype=torch.int64, device=dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    xy = torch.empty((nreq, 2), dtype=torch.float64, device=dev)
    tile = torch.empty((nreq, 2), dtype=torch.int32, device=dev)
    flags = torch.empty(nreq, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    lib = hloc.load_library()
    P = ctypes.c_void_p
    args = (db._h, P(q.data_ptr()), nq, k, w.n_reg, P(offs.data_ptr()), nreq, hloc.FP32,
            P(idx.data_ptr()), P(dist.data_ptr()), P(xy.data_ptr()), P(tile.data_ptr()),
            P(flags.data_ptr()), P(stream.cuda_stream))

    def step():
        rc = lib.hloc_query_batch_async(*args)
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    regions = db.last_regions()
    info = db.info()
    sizes = np.bincount(w.region_of, minlength=w.n_regions_total)
    unique_rows = int(sizes[np.unique(regions)].sum())
    d = w.feats.shape[1]
    screen_bytes = unique_rows * (4 * d + 4) + info["candidates"] * 8 + nq * 4 * d

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    db.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = db.profile_read()
    db.profile(False)
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    screen_ms = phases["screen"][0] / max(phases["screen"][1], 1)
    achieved = screen_bytes / (screen_ms * 1e-3) / 1e9
    gpu_idx = idx.cpu().numpy()

    base, recall, exact, m = (None, None, None, 0)
    if not a.no_cpu_baseline:
        base, recall, exact, m = cpu_baseline(w, gpu_idx, a.cpu_seconds)
    out = {
        "metric": METRIC,
        "value": nq * a.steps / wall,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": int(len(w.feats)), "d": int(d),
                   "regions": int(w.n_regions_total), "frames_per_step": int(nq),
                   "requests_per_step": int(nreq), "n_regions": int(w.n_reg), "k": int(k),
                   "screen": "fp32", "aggregation": list(w.agg)},
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "recall_at_k": recall,
        "exact_lists": None if base is None else f"{exact}/{m}",
        "roofline": {"bound": "hbm", "kernel": "k_screen_f32<false>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": int(screen_bytes),
                     "avg_launch_ms": screen_ms},
        "phases_ms": {p: v[0] / max(v[1], 1) for p, v in phases.items()},
        "fallbacks": {"coarse": info["coarse_fallbacks"], "fine": info["fine_fallbacks"]},
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    db.close()


if __name__ == "__main__":
    main()
