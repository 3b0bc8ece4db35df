#!/usr/bin/env python3
"""Localization throughput of the hloc hot path on one MI355X.

One step = one batch of query frames through the whole path: query prep,
coarse screen and FP64 region re-score, region scheduling, fine MFMA screen,
selection, FP64 rerank, and per-request aggregation, with inputs resident in
device memory. The default workload is the plain-FP32 shape: N = 200,000 rows
of D = 256, 1,024 regions of uneven size, 256 single-frame queries per batch,
8 regions per frame, k = 16.

Throughput is taken over K back-to-back steps, the faster of two ways of
issuing them: one stream with direct launches, or W captured batches (HIP
graphs on W workspaces) replayed round-robin on W streams, whose outputs are
checked bit for bit against the direct run.

Prints one JSON line: throughput (frames/s) of K back-to-back steps, the
host-to-host latency p50/p99 of single batches, the roofline of the fine screen
(algorithmic bytes over its duration from HIP start/stop events in a second
loop of K steps, against HBM peak), and the FP64 oracle timed on a bounded
sample on the host.
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
    """Time the FP64 oracle on the batch's frames, repeating the batch until
    about `seconds` of single-threaded work, and check the GPU's lists on the
    frames it covered."""
    import oracle
    done, passes, t_total = 0, 0, 0.0
    m = min(len(w.q), 8)
    ora = None
    while t_total < seconds:
        t0 = time.perf_counter()
        res = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, w.q[:m], w.k, w.n_reg)
        offs = w.req_offsets
        for r in range(len(offs) - 1):
            if offs[r + 1] > m:
                break
            oracle.aggregate(res["idx"][offs[r]:offs[r + 1]].ravel(), w.xy, *w.agg)
        dt = time.perf_counter() - t0
        t_total += dt
        done += m
        passes += 1
        if ora is None or m > len(ora["idx"]):
            ora = res
        if m < len(w.q):
            m = min(len(w.q), max(m + 1, int(m * (seconds - t_total) / max(dt, 1e-3))))
    mm = len(ora["idx"])
    hits = sum(len(set(gpu_idx[i].tolist()) & set(ora["idx"][i].tolist())) for i in range(mm))
    exact = sum(int(np.array_equal(gpu_idx[i], ora["idx"][i])) for i in range(mm))
    return dict(value=done / t_total, unit="queries/s", cores=1, kind="oracle",
                sample=f"{done} frames of {w.name} ({passes} passes over the first {mm} of "
                       f"{len(w.q)} frames), single thread, {t_total:.1f} s"), \
        hits / (mm * w.k), exact, mm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", type=int, default=1, help="index of workload.SHAPES")
    ap.add_argument("--nq", type=int, default=None, help="override the batch size")
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32",
                    help="fine-screen precision (the rerank is FP64 either way)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--workspaces", type=int, default=2,
                    help="batches in flight in the pipelined loop (one workspace and stream each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (reference for "
                         "hardware byte counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_08861_amd import hloc, workload

    dev = torch.device("cuda:0")
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": a.copy_calibration, "launches": 10}))
        return
    t0 = time.perf_counter()
    w = workload.make_workload(a.workload, nq=a.nq)
    log(f"[bench] workload {w.name}: n={len(w.feats)} d={w.feats.shape[1]} "
        f"regions={w.n_regions_total} frames={len(w.q)} requests={len(w.req_offsets) - 1} "
        f"({time.perf_counter() - t0:.1f} s)")
    db = hloc.HlocDB(w.feats, w.xy, mirrors=hloc.MIRROR_BF16 if a.precision == "bf16" else 0)
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
    args = (db._h, P(q.data_ptr()), nq, k, w.n_reg, P(offs.data_ptr()), nreq,
            hloc.PRECISIONS[a.precision],
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
    row_bytes = 2 * d if a.precision == "bf16" else 4 * d
    screen_bytes = unique_rows * (row_bytes + 4) + info["candidates"] * 8 + nq * row_bytes

    # throughput: K back-to-back steps, nothing recorded between kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    wall_eager = wall
    eager_out = {k_: v.clone() for k_, v in dict(idx=idx, dist=dist, xy=xy, tile=tile,
                                                 flags=flags).items()}
    # pipelined: W workspaces, each holding the captured batch (a HIP graph)
    # and its own outputs, replayed round-robin on W streams so that up to W
    # batches overlap on the device
    W = max(1, a.workspaces)
    wss = [hloc.Workspace(db) for _ in range(W)]
    outs = [hloc.Workspace.outputs(nq, nreq, k, dev) for _ in range(W)]
    streams = [torch.cuda.Stream(dev) for _ in range(W)]
    for ws, o in zip(wss, outs):
        ws.capture(q, k, w.n_reg, offs, o, precision=a.precision)
    torch.cuda.synchronize()
    for i in range(a.warmup):
        wss[i % W].replay(streams[i % W])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        wss[i % W].replay(streams[i % W])
    torch.cuda.synchronize()
    wall_pipe = time.perf_counter() - t0
    for o in outs:
        for key in eager_out:
            if o[key].cpu().numpy().tobytes() != eager_out[key].cpu().numpy().tobytes():
                raise RuntimeError(f"pipelined batch differs from the eager batch in {key}")
    wall = min(wall_eager, wall_pipe)
    # the same K steps again with every kernel dispatched with HIP start/stop
    # events on the query stream: per-phase device time for the roofline (the
    # events add dispatch gaps, so this loop is not used for the throughput)
    db.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t1
    phases = db.profile_read()
    db.profile(False)
    # latency: one batch at a time, host to host
    lat = []
    for _ in range(a.latency_reps):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)
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
        "dtype": "f32" if a.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "n": int(len(w.feats)), "d": int(d),
                   "regions": int(w.n_regions_total), "frames_per_step": int(nq),
                   "requests_per_step": int(nreq), "n_regions": int(w.n_reg), "k": int(k),
                   "screen": a.precision, "rerank": "f64", "aggregation": list(w.agg)},
        "pipeline": {"workspaces": W, "graphs": True, "value_from": "eager" if wall == wall_eager else "pipelined"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency": f"host-to-host time of one batch, {len(lat)} batches run one at a time",
        "recall_at_k": recall,
        "exact_lists": None if base is None else f"{exact}/{m}",
        "roofline": {"bound": "hbm",
                     "kernel": "k_screen_bf16<NS,false>" if a.precision == "bf16" else "k_screen_blk<NS,false>",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": int(screen_bytes),
                     "avg_launch_ms": screen_ms},
        "phases_ms": {p: v[0] / max(v[1], 1) for p, v in phases.items()},
        "ms_per_step_event_timed": wall_prof * 1e3 / a.steps,
        "modes": {"eager_one_stream_ms_per_step": wall_eager * 1e3 / a.steps,
                  f"graphs_{W}_streams_ms_per_step": wall_pipe * 1e3 / a.steps},
        "fallbacks": {"coarse": info["coarse_fallbacks"], "fine": info["fine_fallbacks"]},
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    for ws in wss:
        ws.close()
    db.close()


if __name__ == "__main__":
    main()
