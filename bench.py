#!/usr/bin/env python3
"""Localization throughput of the hloc hot path on one MI355X.

One step = one batch of query frames through the whole path: query prep,
coarse screen and FP64 region re-score, region scheduling, fine MFMA screen,
selection, FP64 rerank, and per-request aggregation, with inputs resident in
device memory. The default workload is the batched multi-frame shape: the
2,000,000 x 512 database with 4,096 lognormal regions, 4,096 requests of 8
frames per batch (32,768 query frames), 8 regions per frame, k = 32, the
paper's aggregation constants, in the form chosen for it (bf16 screen, FP64
rerank); --workload picks another shape of workload.SHAPES.

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
import dataclasses
import ctypes
import csv
import hashlib
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
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # dense, per screen dtype


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the fine screen's sources: hardware counters taken on it stay valid while
# these files are unchanged
SCREEN_SOURCES = ("paper_2006_08861_amd/csrc/screen_f32.hip",
                  "paper_2006_08861_amd/csrc/screen_lp.hip",
                  "paper_2006_08861_amd/csrc/hloc_device.h",
                  "paper_2006_08861_amd/csrc/hloc_internal.h")
# name prefixes of the narrow-item list kernels (their names end in ", false>":
# not dense) and of the wide-item kernels
SCREEN_KERNELS = {"fp32": "k_screen_blk<", "bf16": "k_screen_lp<1, ", "fp8": "k_screen_lp<2, "}
WIDE_KERNELS = {"fp32": "k_screen_wide<", "bf16": "k_screen_wide_rs<1, ", "fp8": "k_screen_wide_rs<2, "}
MIRRORS = {"fp32": lambda h: 0, "bf16": lambda h: h.MIRROR_BF16, "fp8": lambda h: h.MIRROR_FP8}
DTYPES = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}


def screen_digest() -> str:
    h = hashlib.sha256()
    for rel in SCREEN_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_path(workload: str, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"counters_screen_{precision}_{workload}.md")


def narrow_label(precision: str, rows_per_item: int) -> str:
    """The narrow-item kernel's template as it runs with these tiles (the fp32
    kernel hoists the frame operand for items of more than 64 rows)."""
    if precision == "fp32":
        return f"k_screen_blk<NS, {'true' if rows_per_item > 64 else 'false'}, false>"
    return SCREEN_KERNELS[precision] + "NS, false>"


def load_traffic(workload: str, precision: str, rows_per_item: int):
    """HBM bytes per launch of the fine screen from the committed counter
    summary: FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    same counter reads for a plain device copy. The summary holds one record
    per rows-per-item tile (the work items, hence the re-reads, depend on it).
    None when there is no record for this workload and tile or the screen's
    sources changed since it was taken."""
    path = counters_path(workload, precision)
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    recs = []
    with open(path) as f:
        for line in f:
            if line.startswith("record: "):
                recs.append(json.loads(line[len("record: "):]))
    if not recs:
        return None, f"{os.path.relpath(path, ROOT)} holds no record line"
    rec = next((r for r in recs if r.get("rows_per_item") == rows_per_item), None)
    if rec is None:
        return None, f"no counters taken with {rows_per_item}-row items"
    if rec["sources"] != screen_digest():
        return None, "screen sources changed since the counters were taken"
    b = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
    return b, os.path.relpath(path, ROOT)


def _kname(r) -> str:
    return r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hloc::", "")


def per_dispatch_kib(path: str, name_prefix: str, counter: str,
                     suffix: str = "", after: tuple[str, str] | None = None) -> tuple[float, int]:
    """Mean counter value (KiB) per dispatch of the kernels whose name starts
    with name_prefix (after an optional namespace) and ends with suffix in a
    rocprofv3 counter CSV. With after = (prefix, suffix), only dispatches
    whose previous dispatch (by Dispatch_Id) of a screen kernel matches it
    count: the fine stage's wide-item launch follows its narrow-item launch,
    while the coarse stage's dense launch of the same wide kernel does not."""
    with open(path) as f:
        rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r.get("Dispatch_Id") or 0))
    vals = []
    prev = ""
    for r in rows:
        name = _kname(r)
        if name.startswith(name_prefix) and name.endswith(suffix):
            if after is None or (prev.startswith(after[0]) and prev.endswith(after[1])):
                vals.append(float(r["Counter_Value"]))
        if "screen" in name:
            prev = name
    if not vals:
        raise SystemExit(f"no {counter} rows for {name_prefix} in {path}")
    return sum(vals) / len(vals), len(vals)


def counters_summary(a) -> None:
    """Prints the markdown counter summary of the fine screen (with the record
    line load_traffic reads) from four rocprofv3 --pmc CSVs: the benchmark's
    FETCH_SIZE and WRITE_SIZE runs (untuned, with the tiles of --tiles) and the
    copy calibration's. The screen is the narrow-item kernel plus the
    wide-item kernel; their per-dispatch counts are added."""
    if not a.tiles:
        raise SystemExit("--counters-summary needs --tiles: the tiles the counted runs used")
    rows = int(a.tiles.split(",")[0])
    fetch_csv, write_csv, cf_csv, cw_csv = a.counters_summary
    narrow = SCREEN_KERNELS[a.precision]
    wide = WIDE_KERNELS[a.precision]
    per = {}
    for name, prefix, suffix, after in (("narrow", narrow, ", false>", None),
                                        ("wide", wide, ">", (narrow, ", false>"))):
        fk, nf = per_dispatch_kib(fetch_csv, prefix, "FETCH_SIZE", suffix, after)
        wk, nw = per_dispatch_kib(write_csv, prefix, "WRITE_SIZE", suffix, after)
        label = narrow_label(a.precision, rows) if name == "narrow" else prefix + "NS>"
        per[name] = (label, fk, nf, wk, nw)
    copy_bytes = a.copy_mib * (1 << 20)
    copy_kernel = "at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add"
    cfk, _ = per_dispatch_kib(cf_csv, copy_kernel, "FETCH_SIZE")
    cwk, _ = per_dispatch_kib(cw_csv, copy_kernel, "WRITE_SIZE")
    fetch_scale = round(copy_bytes / 1024.0 / cfk, 3)
    write_scale = round(copy_bytes / 1024.0 / cwk, 3)
    fk = sum(v[1] for v in per.values())
    wk = sum(v[3] for v in per.values())
    traffic = 1024.0 * (fk * fetch_scale + wk * write_scale)
    rec = dict(kernel=" + ".join(v[0] for v in per.values()), workload=a.workload_name,
               rows_per_item=rows, tiles=a.tiles, fetch_kib=round(fk, 1), write_kib=round(wk, 1),
               fetch_scale=fetch_scale, write_scale=write_scale, sources=screen_digest())
    if a.counters_append:
        print(f"\n## Tiles {a.tiles} (rows per item, blocks per compute unit)\n")
    else:
        print(f"# Fine-screen HBM traffic, {a.precision} screen, {a.workload_name}\n")
        print("One section per tile choice; the benchmark reads the record line of the "
              "rows-per-item tile it runs with.\n")
        print(f"## Tiles {a.tiles} (rows per item, blocks per compute unit)\n")
    print("Commands (from the repository root, one counter per run):\n")
    print("```")
    for c in a.commands:
        print(c)
    print("```\n")
    print(f"Copy calibration: a {a.copy_mib} MiB device copy reads {cfk:.0f} KiB by FETCH_SIZE "
          f"(scale x{fetch_scale}) and writes {cwk:.0f} KiB by WRITE_SIZE (scale x{write_scale}).\n")
    print("| Kernel | Dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | Bytes per dispatch (scaled) |")
    print("|---|---|---|---|---|")
    for kname, f_, nf, w_, nw in per.values():
        print(f"| `{kname}` | {nf} | {f_:.1f} | {w_:.1f} | "
              f"{1024 * (f_ * fetch_scale + w_ * write_scale) / 1e6:.2f} MB |")
    print(f"\nHBM traffic per screen step (both kernels): {traffic / 1e6:.2f} MB.\n")
    print("record: " + json.dumps(rec))


def oracle_threads() -> int:
    """Host threads for the oracle's pool: the CPUs this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, gpu_idx, seconds: float, sample_frames: int = 256, full_rows: int = 200_000):
    """Time the FP64 oracle as it stands on the host. Databases of up to
    200,000 rows: the whole batch; larger ones: a fixed sample, the first
    whole requests holding at least `sample_frames` frames. The sample is
    retrieved and its requests aggregated once single-threaded and then on a
    pool of threads (the oracle's array work releases the GIL), each repeated
    until about `seconds` of wall time; throughput is frames per second (the
    queries/s unit). The region means are the database's, computed once
    before timing (the library computes them at set_regions). Also checks the
    GPU's lists on the sample."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    offs = np.asarray(w.req_offsets)
    if len(w.feats) <= full_rows:
        nreq = len(offs) - 1
    else:
        nreq = int(np.searchsorted(offs, sample_frames))
        nreq = min(len(offs) - 1, max(1, nreq))
    m = int(offs[nreq])
    q = w.q[:m]
    reps, _ = oracle.region_means(w.feats, w.region_of, w.n_regions_total)

    def work(sl):
        res = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, q[sl], w.k, w.n_reg,
                              reps=reps)
        return res["idx"]

    def aggregate_all(idx):
        for r in range(nreq):
            oracle.aggregate(idx[offs[r]:offs[r + 1]].ravel(), w.xy, *w.agg)

    def timed(threads):
        t0, passes, idx = time.perf_counter(), 0, None
        while True:
            if threads == 1:
                idx = work(slice(0, m))
            else:
                parts = [slice(i, min(m, i + 8)) for i in range(0, m, 8)]
                with ThreadPoolExecutor(threads) as ex:
                    idx = np.concatenate(list(ex.map(work, parts)))
            aggregate_all(idx)
            passes += 1
            dt = time.perf_counter() - t0
            if dt >= seconds / 2 or passes >= 1000:
                return m * passes / dt, passes, dt, idx

    single, p1, t1, ora_idx = timed(1)
    threads = oracle_threads()
    pooled, p2, t2, _ = timed(threads) if threads > 1 else (single, p1, t1, None)
    hits = sum(len(set(gpu_idx[i].tolist()) & set(ora_idx[i].tolist())) for i in range(m))
    exact = sum(int(np.array_equal(gpu_idx[i], ora_idx[i])) for i in range(m))
    what = "every frame of the batch" if m == len(w.q) else \
        f"a fixed sample: the first {nreq} requests ({m} frames) of the batch"
    return dict(value=pooled, unit="queries/s", cores=threads, kind="oracle",
                single_core_value=single,
                sample=f"{what} of {w.name}; {p1} passes single-threaded in {t1:.1f} s, "
                       f"{p2} passes on {threads} threads in {t2:.1f} s"), \
        hits / (m * w.k), exact, m


FFT_SOURCE = "paper_2006_08861_amd/csrc/fft.hip"
FFT_KERNEL = "k_fft_magnitude"


def fft_kernel_name(length: int) -> str:
    """The kernel a launch of this signal length runs (four-step for L = 128
    and 512, radix-2 in LDS otherwise)."""
    return {128: "k_fft_magnitude_sq<8>", 512: "k_fft_magnitude_sq<16>"}.get(length, FFT_KERNEL)


def fft_digest() -> str:
    with open(os.path.join(ROOT, FFT_SOURCE), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def fft_workload_name(nsig: int, length: int, bins: int) -> str:
    return f"fft-{nsig // 1000}k-L{length}-d{bins}" if nsig % 1000 == 0 else \
        f"fft-{nsig}-L{length}-d{bins}"


def fft_counters_path(name: str) -> str:
    return os.path.join(ROOT, "profiles", f"counters_fft_{name}.md")


def load_fft_traffic(name: str):
    """HBM bytes per launch of the feature kernel from its committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the copy
    calibration), or None when there is none or the kernel changed since."""
    path = fft_counters_path(name)
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    with open(path) as f:
        recs = [json.loads(l[len("record: "):]) for l in f if l.startswith("record: ")]
    if not recs:
        return None, f"{os.path.relpath(path, ROOT)} holds no record line"
    rec = recs[-1]
    if rec["sources"] != fft_digest():
        return None, "the kernel's source changed since the counters were taken"
    b = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
    return b, os.path.relpath(path, ROOT)


def fft_counters_summary(a) -> None:
    """Markdown counter summary of the feature kernel (with the record line
    load_fft_traffic reads) from four rocprofv3 --pmc CSVs: the FETCH_SIZE and
    WRITE_SIZE runs of `bench.py --fft` and the copy calibration's."""
    fetch_csv, write_csv, cf_csv, cw_csv = a.fft_counters
    name = fft_workload_name(a.fft_signals, a.fft_len, a.fft_bins)
    kname = fft_kernel_name(a.fft_len)
    fk, nf = per_dispatch_kib(fetch_csv, kname, "FETCH_SIZE")
    wk, nw = per_dispatch_kib(write_csv, kname, "WRITE_SIZE")
    copy_bytes = a.copy_mib * (1 << 20)
    copy_kernel = "at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add"
    cfk, _ = per_dispatch_kib(cf_csv, copy_kernel, "FETCH_SIZE")
    cwk, _ = per_dispatch_kib(cw_csv, copy_kernel, "WRITE_SIZE")
    fetch_scale = round(copy_bytes / 1024.0 / cfk, 3)
    write_scale = round(copy_bytes / 1024.0 / cwk, 3)
    algo = a.fft_signals * 4 * (a.fft_len + a.fft_bins)
    traffic = 1024.0 * (fk * fetch_scale + wk * write_scale)
    rec = dict(kernel=kname, workload=name, fetch_kib=round(fk, 1), write_kib=round(wk, 1),
               fetch_scale=fetch_scale, write_scale=write_scale, sources=fft_digest())
    print(f"# Feature-kernel HBM traffic, {name}\n")
    print("Commands (from the repository root, one counter per run):\n")
    print("```")
    for c in a.commands:
        print(c)
    print("```\n")
    print(f"Copy calibration: a {a.copy_mib} MiB device copy reads {cfk:.0f} KiB by FETCH_SIZE "
          f"(scale x{fetch_scale}) and writes {cwk:.0f} KiB by WRITE_SIZE (scale x{write_scale}).\n")
    print("| Kernel | Dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | Bytes per dispatch (scaled) "
          "| Algorithmic bytes |")
    print("|---|---|---|---|---|---|")
    print(f"| `{kname}` | {min(nf, nw)} | {fk:.1f} | {wk:.1f} | {traffic / 1e6:.2f} MB | "
          f"{algo / 1e6:.2f} MB |\n")
    print("record: " + json.dumps(rec))


def fft_bench(a) -> None:
    """Fourier-magnitude features of a database's worth of panoramic signals
    (default 200,000 signals of 512 samples to 256 bins: the rows of
    fp32-200k-d256), resident in HBM. A step is one launch over all signals."""
    import torch
    from threadpoolctl import threadpool_limits

    import oracle
    from paper_2006_08861_amd import hloc, workload

    nsig, L, d = a.fft_signals, a.fft_len, a.fft_bins
    name = fft_workload_name(nsig, L, d)
    dev = torch.device("cuda:0")
    x_h = workload.panoramic_signals(nsig, L, np.random.default_rng(2006))
    x = torch.from_numpy(x_h).to(dev)
    out = torch.empty((nsig, d), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    lib = hloc.load_library()
    P = ctypes.c_void_p
    args = (P(x.data_ptr()), nsig, L, d, P(out.data_ptr()), P(stream.cuda_stream))

    def step():
        rc = lib.hloc_fft_features_async(*args)
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = e0.elapsed_time(e1) / a.steps
    algo = nsig * 4 * (L + d)
    achieved = algo / (launch_ms * 1e-3) / 1e9
    traffic, traffic_src = load_fft_traffic(name)

    # parity on seeded sample rows against the oracle (relative to each
    # row's largest bin)
    got = out.cpu().numpy()
    rows = np.sort(np.random.default_rng(2007).choice(nsig, min(nsig, 512), replace=False))
    ora = oracle.fft_magnitude(x_h[rows], d)
    rel = float((np.abs(got[rows] - ora) / ora.max(axis=1, keepdims=True)).max())
    equal = float(np.mean(got[rows] == ora.astype(np.float32)))

    base = None
    if not a.no_cpu_baseline:
        done, t_cpu, m = 0, 0.0, 256
        with threadpool_limits(limits=1):
            while t_cpu < a.cpu_seconds:
                lo = done % nsig
                t1 = time.perf_counter()
                oracle.fft_magnitude(x_h[lo:lo + m], d)
                t_cpu += time.perf_counter() - t1
                done += len(x_h[lo:lo + m])
        base = dict(value=done / t_cpu, unit="signals/s", cores=1, kind="oracle",
                    sample=f"{done} signals of {name} in chunks of {m}, DFT by its definition "
                           f"(FP64 matrix product), single thread, {t_cpu:.1f} s")
    print(json.dumps({
        "metric": "omnidirectional features/s (Fourier magnitude, FP64, rounded to fp32) vs "
                  "FP64 oracle; HBM GB/s % peak",
        "value": nsig * a.steps / wall, "unit": "signals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wall * 1e3 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "signals": nsig, "len": L, "bins": d},
        "roofline": {"bound": "hbm", "kernel": fft_kernel_name(L), "achieved": achieved, "peak": 8000.0,
                     "unit": "GB/s", "frac": achieved / 8000.0, "traffic": traffic,
                     "traffic_source": traffic_src, "bytes_per_launch": algo,
                     "avg_launch_ms": launch_ms},
        "parity": {"sample_rows": int(len(rows)), "max_err_rel_row_max": rel,
                   "equal_to_rounded_oracle": equal},
        "cpu_baseline": base}), flush=True)


def windows_bench(a) -> None:
    """Sliding-window requests over a video along the walk of fp32-200k-d256:
    T frames (consecutive database rows plus N(0, 0.1^2) noise), one request
    per window of M consecutive frames (Section 4 uses M = 11). Each frame is
    retrieved once and every window pools its frames' lists
    (hloc_query_windows_async); the same windows sent as materialised
    requests (every window's M frames again) are timed beside it."""
    import torch

    import oracle
    from paper_2006_08861_amd import hloc, workload

    w = workload.make_workload(1)
    rng = np.random.default_rng(2016)
    T, M = a.windows_frames, a.windows
    s0 = int(rng.integers(0, len(w.feats) - T))
    q_h = (w.feats[s0:s0 + T] + 0.1 * rng.standard_normal((T, w.feats.shape[1]))).astype(np.float32)
    nreq = T - M + 1
    frames_h = np.concatenate([np.arange(i, i + M) for i in range(nreq)]).astype(np.int32)
    offs_h = (np.arange(nreq + 1) * M).astype(np.int32)
    agg = (0.3, 10, 3.0, 20)
    name = f"{w.name}-video{T}-window{M}"
    dev = torch.device("cuda:0")
    db = hloc.HlocDB(w.feats, w.xy)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*agg)
    k, n_reg = w.k, w.n_reg
    q, frames, offs = (torch.from_numpy(x).to(dev) for x in (q_h, frames_h, offs_h))
    qm = q[frames.long()].contiguous()
    db.reserve(len(frames_h), nreq, k, n_reg)
    stream = torch.cuda.current_stream(dev)
    lib = hloc.load_library()
    P = ctypes.c_void_p
    o = {"idx": torch.empty((T, k), dtype=torch.int64, device=dev),
         "dist": torch.empty((T, k), dtype=torch.float32, device=dev),
         "xy": torch.empty((nreq, 2), dtype=torch.float64, device=dev),
         "tile": torch.empty((nreq, 2), dtype=torch.int32, device=dev),
         "flags": torch.empty(nreq, dtype=torch.int32, device=dev)}
    om = dict(o, idx=torch.empty((len(frames_h), k), dtype=torch.int64, device=dev),
              dist=torch.empty((len(frames_h), k), dtype=torch.float32, device=dev),
              xy=torch.empty_like(o["xy"]), tile=torch.empty_like(o["tile"]),
              flags=torch.empty_like(o["flags"]))
    outp = lambda d: tuple(P(d[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags"))

    def step_windows():
        rc = lib.hloc_query_windows_async(db._h, P(q.data_ptr()), T, k, n_reg, P(offs.data_ptr()),
                                          P(frames.data_ptr()), len(frames_h), nreq, hloc.FP32,
                                          *outp(o), P(stream.cuda_stream))
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    def step_materialised():
        rc = lib.hloc_query_batch_async(db._h, P(qm.data_ptr()), len(frames_h), k, n_reg,
                                        P(offs.data_ptr()), nreq, hloc.FP32, *outp(om),
                                        P(stream.cuda_stream))
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    def timed(step):
        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / a.steps

    t_win = timed(step_windows)
    t_mat = timed(step_materialised)
    for key in ("xy", "tile", "flags"):
        if o[key].cpu().numpy().tobytes() != om[key].cpu().numpy().tobytes():
            raise RuntimeError(f"windows and materialised requests differ in {key}")
    # the fine screen of the windows batch, event-timed per dispatch
    db.profile(True)
    for _ in range(a.steps):
        step_windows()
    torch.cuda.synchronize()
    phases = db.profile_read()
    db.profile(False)
    info = db.info()
    regions = db.last_regions()
    sizes = np.bincount(w.region_of, minlength=w.n_regions_total)
    d = w.feats.shape[1]
    screen_bytes = int(sizes[np.unique(regions)].sum()) * (4 * d + 4) + info["candidates"] * 4 \
        + T * 4 * d
    screen_ms = phases["screen"][0] / max(phases["screen"][1], 1)
    if info["items"] > info["narrow_items"]:
        screen_ms += phases["screen_wide"][0] / max(phases["screen_wide"][1], 1)
    achieved = screen_bytes / (screen_ms * 1e-3) / 1e9
    # oracle on the first windows (their frames retrieved once), about a.cpu_seconds
    base, same = None, None
    if not a.no_cpu_baseline:
        m, t_cpu, done = 4, 0.0, 0
        while t_cpu < a.cpu_seconds and m <= nreq:
            t1 = time.perf_counter()
            ora = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, q_h[:m + M - 1],
                                  offs_h[:m + 1], k, n_reg, agg, req_frames=frames_h[:m * M])
            t_cpu += time.perf_counter() - t1
            done += m
            tile = o["tile"].cpu().numpy()[:m]
            same = (int((tile == ora["tile"]).all(axis=1).sum()), m)
            m *= 2
        base = dict(value=done / t_cpu, unit="requests/s", cores=1, kind="oracle",
                    sample=f"{done} windows of {name} (the first 4, 8, ... windows, each set "
                           f"retrieving its frames once), single thread, {t_cpu:.1f} s")
    print(json.dumps({
        "metric": "sliding-window localization requests/s (frames retrieved once, windows "
                  "pooled) vs FP64 oracle; HBM GB/s % peak",
        "value": nreq / t_win, "unit": "requests/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": t_win * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "frames": T, "window": M, "requests": nreq, "k": k,
                   "n_regions": n_reg, "aggregation": list(agg)},
        "materialised": {"requests_per_s": nreq / t_mat, "ms_per_step": t_mat * 1e3,
                         "frames_screened": int(len(frames_h))},
        "speedup_vs_materialised": t_mat / t_win,
        "same_tiles_as_oracle": None if same is None else f"{same[0]}/{same[1]}",
        "roofline": {"bound": "hbm", "kernel": "fine screen (narrow + wide items)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": screen_bytes, "avg_launch_ms": screen_ms},
        "cpu_baseline": base}), flush=True)
    db.close()


def labels_bench(a) -> None:
    """Top N per (frame, path) with Section 4's parameters on fp32-200k-d256:
    the 1,024 regions split into P contiguous runs (walked paths), requests
    of M = 11 consecutive frames of the batch, N = 15 per frame and path, so
    a request pools N x M x P = 825 candidates at P = 5."""
    import torch

    import oracle
    from paper_2006_08861_amd import hloc, workload

    w = workload.make_workload(1)
    P, M, k = a.labels, 11, 15
    R = w.n_regions_total
    labels = ((np.arange(R) * P) // R).astype(np.int32)
    nq = (len(w.q) // M) * M
    q_h = w.q[:nq]
    offs_h = np.arange(0, nq + 1, M).astype(np.int32)
    nreq = len(offs_h) - 1
    agg = (0.3, 10, 3.0, 20)
    name = f"{w.name}-paths{P}-window{M}-top{k}"
    dev = torch.device("cuda:0")
    db = hloc.HlocDB(w.feats, w.xy)
    db.set_regions(w.region_of, R)
    db.set_aggregation(*agg)
    db.set_region_labels(labels, P)
    db.reserve(nq, nreq, k, w.n_reg)
    q = torch.from_numpy(q_h).to(dev)
    offs = torch.from_numpy(offs_h).to(dev)
    out = {"idx": torch.empty((P, nq, k), dtype=torch.int64, device=dev),
           "dist": torch.empty((P, nq, k), dtype=torch.float32, device=dev),
           "xy": torch.empty((nreq, 2), dtype=torch.float64, device=dev),
           "tile": torch.empty((nreq, 2), dtype=torch.int32, device=dev),
           "flags": torch.empty(nreq, dtype=torch.int32, device=dev)}
    stream = torch.cuda.current_stream(dev)
    lib = hloc.load_library()
    Pp = ctypes.c_void_p
    args = (db._h, Pp(q.data_ptr()), nq, k, w.n_reg, P, Pp(offs.data_ptr()), nreq, hloc.FP32,
            *(Pp(out[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags")),
            Pp(stream.cuda_stream))

    def step():
        rc = lib.hloc_query_labels_async(*args)
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / a.steps
    # the fine screen, event-timed: with n_regions within every path's
    # regions the paths run as one batch of frames x paths (one screen launch)
    db.profile(True)
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    phases = db.profile_read()
    db.profile(False)
    info = db.info()
    regions = db.last_regions()
    sizes = np.bincount(w.region_of, minlength=R)
    d = w.feats.shape[1]
    screen_bytes = int(sizes[np.unique(regions)].sum()) * (4 * d + 4) + info["candidates"] * 4 \
        + nq * 4 * d
    screen_ms = phases["screen"][0] / max(phases["screen"][1], 1)
    if info["items"] > info["narrow_items"]:
        screen_ms += phases["screen_wide"][0] / max(phases["screen_wide"][1], 1)
    achieved = screen_bytes / (screen_ms * 1e-3) / 1e9
    base, same = None, None
    if not a.no_cpu_baseline:
        m, t_cpu, done = 1, 0.0, 0
        tile = out["tile"].cpu().numpy()
        while t_cpu < a.cpu_seconds and m <= nreq:
            t1 = time.perf_counter()
            ora = oracle.localize_labels(w.feats, w.xy, w.region_of, R, labels, q_h[:m * M],
                                         offs_h[:m + 1], k, w.n_reg, agg)
            t_cpu += time.perf_counter() - t1
            done += m
            same = (int((tile[:m] == ora["tile"]).all(axis=1).sum()), m)
            m *= 2
        base = dict(value=done / t_cpu, unit="requests/s", cores=1, kind="oracle",
                    sample=f"{done} requests of {name} (the first 1, 2, 4, ... requests), "
                           f"single thread, {t_cpu:.1f} s")
    print(json.dumps({
        "metric": "localization requests/s with top-N per (frame, path) pooled (N x M x P "
                  "candidates) vs FP64 oracle; HBM GB/s % peak",
        "value": nreq / wall, "unit": "requests/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "paths": P, "frames_per_request": M, "top_n": k,
                   "requests": nreq, "frames": nq, "candidates_per_request": k * M * P,
                   "n_regions": w.n_reg, "aggregation": list(agg)},
        "same_tiles_as_oracle": None if same is None else f"{same[0]}/{same[1]}",
        "roofline": {"bound": "hbm", "kernel": "fine screen (frames x paths in one batch)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": screen_bytes, "avg_launch_ms": screen_ms},
        "cpu_baseline": base}), flush=True)
    db.close()


def streams_bench(a) -> None:
    """Sliding windows across calls (hloc_query_streams_async) on
    fp32-200k-d256: a.streams_n video streams along the walk (consecutive
    rows plus N(0, 0.1^2) noise), each call bringing one new frame per
    stream; every frame's window is the frame and the a.streams - 1 before it
    in its stream, kept on the device between calls. Value: window estimates
    (frames) per second over a.steps calls."""
    import torch

    from paper_2006_08861_amd import hloc, workload

    w = workload.make_workload(1)
    S, M = a.streams_n, a.streams
    T = a.warmup + a.steps
    rng = np.random.default_rng(2016)
    starts = rng.integers(0, len(w.feats) - T, S)
    d = w.feats.shape[1]
    q_h = np.stack([w.feats[starts + t] for t in range(T)]).astype(np.float32)
    q_h += (0.1 * rng.standard_normal(q_h.shape)).astype(np.float32)
    agg = (0.3, 10, 3.0, 20)
    dev = torch.device("cuda:0")
    db = hloc.HlocDB(w.feats, w.xy)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*agg)
    k, n_reg = w.k, w.n_reg
    st = hloc.Streams(db, S, M, k, max_frames=S)
    q = torch.from_numpy(q_h).to(dev)
    offs = torch.arange(S + 1, dtype=torch.int32, device=dev)
    sid = torch.arange(S, dtype=torch.int32, device=dev)
    o = {"idx": torch.empty((S, k), dtype=torch.int64, device=dev),
         "dist": torch.empty((S, k), dtype=torch.float32, device=dev),
         "xy": torch.empty((S, 2), dtype=torch.float64, device=dev),
         "tile": torch.empty((S, 2), dtype=torch.int32, device=dev),
         "flags": torch.empty(S, dtype=torch.int32, device=dev)}
    lib = hloc.load_library()
    P = ctypes.c_void_p
    stream = torch.cuda.current_stream(dev)
    outp = tuple(P(o[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags"))

    def call(t):
        rc = lib.hloc_query_streams_async(st._h, P(q[t].data_ptr()), S, n_reg, hloc.FP32,
                                          P(offs.data_ptr()), P(sid.data_ptr()), S, *outp,
                                          P(stream.cuda_stream))
        if rc != 0:
            raise hloc.HlocError(rc, lib.hloc_last_error().decode())

    for t in range(a.warmup):
        call(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(a.warmup, T):
        call(t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st.close()
    db.close()
    print(json.dumps({
        "metric": "window estimates/s (sliding windows across calls, one new frame per stream "
                  "per call)",
        "value": S * a.steps / wall, "unit": "frames/s", "ms_per_call": wall * 1e3 / a.steps,
        "steps": a.steps, "warmup": a.warmup, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}-streams{S}-window{M}", "streams": S, "window": M,
                   "k": k, "n_regions": n_reg}}), flush=True)


def serve_bench(a) -> None:
    """Poisson arrivals of 1-16 frame requests (k in {8, 16, 32}) into the
    request server, at each rate of a.serve (requests/s, comma-separated) for
    a.serve_seconds; one database, a fresh server per rate; prints one JSON
    line per rate with the completed rate, the submit-to-completion latency
    and the refused requests."""
    import queue
    import threading

    import torch  # noqa: F401
    from paper_2006_08861_amd import hloc, workload

    t0 = time.perf_counter()
    w = workload.make_workload(4, n=a.serve_n)
    log(f"[serve] workload {w.name}: n={len(w.feats)} d={w.feats.shape[1]} "
        f"regions={w.n_regions_total} request pool={len(w.req_offsets) - 1} "
        f"({time.perf_counter() - t0:.1f} s)")
    db = hloc.HlocDB(w.feats, w.xy, mirrors=MIRRORS[a.precision](hloc))
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    offs = w.req_offsets
    npool = len(offs) - 1
    pool = [np.ascontiguousarray(w.q[offs[r]:offs[r + 1]]) for r in range(npool)]
    for rate in (float(v) for v in str(a.serve).split(",")):
        srv = hloc.Server(db, k=32, n_regions=w.n_reg, precision=a.precision,
                          max_batch_frames=a.serve_batch, max_slots=a.workspaces,
                          max_queue_frames=a.serve_queue, hbm_budget_bytes=a.serve_budget)
        rng = np.random.default_rng(77)
        n_req = int(rate * a.serve_seconds)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        pick = rng.integers(0, npool, n_req)
        ks = rng.choice([8, 16, 32], n_req)
        # warm-up: one request of every size
        for f in range(1, 17):
            r = next(i for i in range(npool) if offs[i + 1] - offs[i] >= f)
            t = srv.submit(pool[r][:f], 32)
            srv.wait(t, f, 32)
        tickets = queue.Queue()
        lat, refused = [], [0]
        done_frames = [0]

        def waiter():
            while True:
                item = tickets.get()
                if item is None:
                    return
                t, nf, k = item
                out = srv.wait(t, nf, k)
                lat.append(out["latency_ms"])
                done_frames[0] += nf

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        for i in range(n_req):
            due = start + arrivals[i]
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 3e-4:
                    time.sleep(due - now - 2e-4)
            frames = pool[pick[i]]
            try:
                t = srv.submit(frames, int(ks[i]))
            except hloc.HlocError as e:
                if e.code != hloc.EBUSY:
                    raise
                refused[0] += 1
                continue
            tickets.put((t, len(frames), int(ks[i])))
        tickets.put(None)
        th.join()
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        lat = np.array(lat)
        print(json.dumps({
            "metric": "served localization requests/s (Poisson arrivals, 1-16 frames, k 8/16/32)",
            "offered_req_per_s": rate, "value": len(lat) / wall, "unit": "requests/s",
            "frames_per_s": done_frames[0] / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "refused": refused[0], "seconds": wall,
            "dtype": DTYPES[a.precision], "data": "synthetic",
            "config": {"workload": w.name, "n": int(len(w.feats)), "d": int(w.feats.shape[1]),
                       "regions": int(w.n_regions_total), "n_regions": int(w.n_reg),
                       "max_batch_frames": a.serve_batch, "slots": st["slots"],
                       "hbm_budget_bytes": a.serve_budget},
            "server": st}), flush=True)
    db.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", type=int, default=3,
                    help="index of workload.SHAPES (default: the multi-frame 2M x 512 shape)")
    ap.add_argument("--nq", type=int, default=None, help="override the batch size")
    ap.add_argument("--n-regions", type=int, default=None,
                    help="override the regions searched per frame (>= the region count: the "
                         "exhaustive search)")
    ap.add_argument("--precision", choices=("fp32", "bf16", "fp8"), default=None,
                    help="fine-screen precision (the rerank is FP64 either way); default: the "
                         "form chosen for the workload (fp32 up to 200,000 rows, bf16 above)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--workspaces", type=int, default=4,
                    help="batches in flight in the pipelined loop (one workspace and stream each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default fine-screen tiles instead of timing the candidates")
    ap.add_argument("--tiles", default=None, metavar="ROWS,BLOCKS",
                    help="use these fine-screen tiles (rows per item, blocks per CU) untuned")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (reference for "
                         "hardware byte counters) and exit")
    ap.add_argument("--counters-summary", nargs=4, metavar="CSV",
                    help="only print the fine screen's counter summary from rocprofv3 --pmc "
                         "CSVs: FETCH_SIZE, WRITE_SIZE, copy FETCH_SIZE, copy WRITE_SIZE")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy size of the calibration CSVs")
    ap.add_argument("--workload-name", default="fp32-200k-d256")
    ap.add_argument("--commands", nargs="*", default=[], help="commands quoted in the summary")
    ap.add_argument("--counters-append", action="store_true",
                    help="print only the section of one more tile choice (appended to a summary)")
    ap.add_argument("--serve", default="", metavar="REQ_PER_S[,...]",
                    help="only run the request server under Poisson arrivals at these rates "
                         "(requests/s, comma-separated: one line each)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-n", type=int, default=None, help="database rows (default: 4M)")
    ap.add_argument("--serve-batch", type=int, default=512, help="frames per batch")
    ap.add_argument("--serve-queue", type=int, default=1 << 16, help="frames waiting at most")
    ap.add_argument("--serve-budget", type=int, default=0, help="HBM bytes for the slots")
    ap.add_argument("--labels", type=int, default=0, metavar="P",
                    help="only run top-N per (frame, path) over P paths (N = 15, M = 11)")
    ap.add_argument("--windows", type=int, default=0, metavar="M",
                    help="only run sliding-window requests of M frames over a video")
    ap.add_argument("--windows-frames", type=int, default=256, help="video frames per batch")
    ap.add_argument("--streams", type=int, default=0, metavar="M",
                    help="only run sliding windows of M frames across calls (hloc_streams)")
    ap.add_argument("--streams-n", type=int, default=256, help="video streams (one frame each per call)")
    ap.add_argument("--fft", action="store_true",
                    help="only time the Fourier-magnitude feature kernel")
    ap.add_argument("--fft-signals", type=int, default=200_000)
    ap.add_argument("--fft-len", type=int, default=512)
    ap.add_argument("--fft-bins", type=int, default=256)
    ap.add_argument("--fft-counters", nargs=4, metavar="CSV",
                    help="only print the feature kernel's counter summary from rocprofv3 --pmc "
                         "CSVs: FETCH_SIZE, WRITE_SIZE, copy FETCH_SIZE, copy WRITE_SIZE")
    a = ap.parse_args()
    if a.fft_counters:
        fft_counters_summary(a)
        return
    if a.labels:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        labels_bench(a)
        return
    if a.windows:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        windows_bench(a)
        return
    if a.fft:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        fft_bench(a)
        return
    if a.streams:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        streams_bench(a)
        return
    if a.serve:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        a.precision = a.precision or "fp32"
        serve_bench(a)
        return
    if a.counters_summary:
        counters_summary(a)
        return
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
    if a.precision is None:
        a.precision = "fp32" if workload.SHAPES[a.workload]["n"] <= 200_000 else "bf16"
    t0 = time.perf_counter()
    w = workload.make_workload(a.workload, nq=a.nq)
    if a.n_regions is not None and a.n_regions != w.n_reg:
        tag = "exhaustive" if a.n_regions >= w.n_regions_total else f"nreg{a.n_regions}"
        w = dataclasses.replace(w, n_reg=a.n_regions, name=f"{w.name}-{tag}")
    log(f"[bench] workload {w.name}: n={len(w.feats)} d={w.feats.shape[1]} "
        f"regions={w.n_regions_total} frames={len(w.q)} requests={len(w.req_offsets) - 1} "
        f"({time.perf_counter() - t0:.1f} s)")
    db = hloc.HlocDB(w.feats, w.xy, mirrors=MIRRORS[a.precision](hloc))
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

    tiles = None
    if a.tiles:
        rows, blocks = (int(v) for v in a.tiles.split(","))
        db.set_tiles(rows, blocks)
    elif not a.no_autotune:
        # fine-screen tiles for this shape, timed on the batch itself
        tiles = db.autotune(q, k, w.n_reg, a.precision, reps=5)
        log(f"[bench] tiles {tiles}")

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
    row_bytes = {"fp32": 4 * d, "bf16": 2 * d, "fp8": d + 4}[a.precision]  # fp8: + scale
    # algorithmic bytes of the fine screen: every row of every region kept by
    # some frame (with its norm) and the frames, each read once; what the
    # screen writes for the select is an intermediate and is not counted
    screen_bytes = unique_rows * (row_bytes + 4) + nq * row_bytes

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
    # latency: one batch at a time, host to host, and on the device (HIP
    # events on the query stream around the batch)
    lat, lat_dev = [], []
    for _ in range(a.latency_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t1 = time.perf_counter()
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
        lat_dev.append(e0.elapsed_time(e1))
    lat, lat_dev = np.array(lat), np.array(lat_dev)
    # the fine screen: the narrow-item kernel, plus the wide-item kernel that
    # follows it when some region is kept by more than 16 frames
    wide_items = info["items"] - info["narrow_items"]
    screen_ms = phases["screen"][0] / max(phases["screen"][1], 1)
    if wide_items > 0:
        screen_ms += phases["screen_wide"][0] / max(phases["screen_wide"][1], 1)
    achieved = screen_bytes / (screen_ms * 1e-3) / 1e9
    # 2 D flops per (frame, row) word: past the dtype's ridge point (all
    # frames against many rows, as in the exhaustive search) the screen is
    # bound by the matrix cores, not by HBM
    screen_flops = 2.0 * info["candidates"] * d
    screen_dtype = a.precision
    mfma_bound = screen_flops / screen_bytes > MFMA_PEAK_TFLOPS[screen_dtype] / (HBM_PEAK_GBS / 1e3)
    traffic, traffic_src = load_traffic(w.name, a.precision, db.tiles()["rows_per_item"])
    # the coarse screen is the dense (GEMM-shaped) part: nq x R distances
    coarse_ms = phases["coarse"][0] / max(phases["coarse"][1], 1)
    s1_flops = 2.0 * nq * w.n_regions_total * d
    s1_tf = s1_flops / (coarse_ms * 1e-3) / 1e12 if coarse_ms > 0 else 0.0
    # fp8 queries screen the representatives in bf16 (bf16 copies are kept
    # beside an fp8 mirror)
    s1_dtype = "bf16" if a.precision == "fp8" else a.precision
    # bf16 coarse screens run as the fused product with its key lists (the
    # frames it defers are timed apart, in the coarse_defer phase)
    fused = s1_dtype == "bf16" and d % 64 == 0 and d <= 512
    stage1 = {"kernel": "k_coarse_gemm<NS, false> (bf16 product, kept-quad epilogue)" if fused
              else "coarse screen (" + ("wide" if nq >= 512 else "narrow") + " kernel, dense)",
              "dtype": s1_dtype, "flops": s1_flops, "avg_launch_ms": coarse_ms, "achieved": s1_tf,
              "peak": MFMA_PEAK_TFLOPS[s1_dtype], "unit": "TFLOP/s",
              "frac": s1_tf / MFMA_PEAK_TFLOPS[s1_dtype]}
    gpu_idx = idx.cpu().numpy()

    base, recall, exact, m = (None, None, None, 0)
    if not a.no_cpu_baseline:
        base, recall, exact, m = cpu_baseline(w, gpu_idx, a.cpu_seconds)
    phase_ms = {p: v[0] / max(v[1], 1) for p, v in phases.items()}
    dominant = max(phase_ms, key=phase_ms.get)
    out = {
        "metric": METRIC,
        "value": nq * a.steps / wall,
        "unit": "queries/s",
        "query": "one query frame retrieved (top k) and pooled into its request's estimate",
        "requests_per_s": nreq * a.steps / wall,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[a.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "n": int(len(w.feats)), "d": int(d),
                   "regions": int(w.n_regions_total), "frames_per_step": int(nq),
                   "requests_per_step": int(nreq), "n_regions": int(w.n_reg), "k": int(k),
                   "screen": a.precision, "rerank": "f64", "aggregation": list(w.agg),
                   "tiles": db.tiles()},
        "pipeline": {"workspaces": W, "graphs": True, "value_from": "eager" if wall == wall_eager else "pipelined"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency": f"host-to-host time of one batch, {len(lat)} batches run one at a time",
        "device_p50_ms": float(np.percentile(lat_dev, 50)),
        "device_p99_ms": float(np.percentile(lat_dev, 99)),
        "recall_at_k": recall,
        "exact_lists": None if base is None else f"{exact}/{m}",
        "roofline": ({"bound": "mfma",
                      "kernel": narrow_label(a.precision, db.tiles()["rows_per_item"])
                                + (" + wide-item kernel" if wide_items > 0 else ""),
                      "achieved": screen_flops / (screen_ms * 1e-3) / 1e12,
                      "peak": MFMA_PEAK_TFLOPS[screen_dtype], "unit": "TFLOP/s",
                      "frac": screen_flops / (screen_ms * 1e-3) / 1e12
                              / MFMA_PEAK_TFLOPS[screen_dtype],
                      "traffic": None if traffic is None else int(traffic),
                      "traffic_source": traffic_src, "flops_per_launch": screen_flops,
                      "bytes_per_launch": int(screen_bytes), "hbm_gbs": achieved,
                      "avg_launch_ms": screen_ms} if mfma_bound else
                     {"bound": "hbm",
                      "kernel": narrow_label(a.precision, db.tiles()["rows_per_item"])
                                + (" + wide-item kernel" if wide_items > 0 else ""),
                      "achieved": achieved,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                      "traffic": None if traffic is None else int(traffic),
                      "traffic_source": traffic_src, "bytes_per_launch": int(screen_bytes),
                      "avg_launch_ms": screen_ms}),
        "stage1_mfma": stage1,
        "phases_ms": phase_ms,
        "dominant_phase": dominant,
        "ms_per_step_event_timed": wall_prof * 1e3 / a.steps,
        "modes": {"eager_one_stream_ms_per_step": wall_eager * 1e3 / a.steps,
                  f"graphs_{W}_streams_ms_per_step": wall_pipe * 1e3 / a.steps},
        "fallbacks": {"coarse": info["coarse_fallbacks"], "coarse_deferred": info["coarse_deferred"],
                      "fine": info["fine_fallbacks"], "chunked_bands": info["chunked_bands"],
                      "band_rows": info["band_rows"], "rerank_rows": info["rerank_rows"]},
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    for ws in wss:
        ws.close()
    db.close()


if __name__ == "__main__":
    main()
