"""Parity at the full sizes of the measured shapes, through the C ABI.

The 2M x 512 database (bf16-2m-d512, and the multi-frame fp8-2m-d512-8frame
shape on the same rows) and the 4M x 256 serving database are built once per
module; every batch runs at its real size (2,048 frames; 4,096 requests of 8
frames; 4,096 requests of 1-16 frames) through every screen precision, which
must agree bit for bit (each ends in the same certified FP64 rerank), and at
least 1,024 sampled frames (whole requests) are judged against the FP64
oracle with the acceptance rule of tests/parity.py. These shapes reach what
only fires at full size: a region of ~19,000 rows kept by more than a
thousand frames, the multi-kernel schedule, 32,768-frame selects and the
wide bands of the fp8 screen.

The oracle runs on a thread pool (its array work releases the GIL), so no
process is forked from one that holds the GPU.
"""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from parity import judge_frames, judge_requests
from paper_2006_08861_amd import hloc, workload

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SAMPLE_FRAMES = 1024
ALL_MIRRORS = hloc.MIRROR_BF16 | hloc.MIRROR_FP8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def pooled_retrieve(w, q, k, reps, chunk=8):
    """oracle.retrieve over the frames of q, in chunks on a thread pool; the
    per-frame results are concatenated in frame order."""
    parts = [slice(i, min(len(q), i + chunk)) for i in range(0, len(q), chunk)]

    def job(sl):
        return oracle.retrieve(w.feats, w.region_of, w.n_regions_total, q[sl], k, w.n_reg,
                               reps=reps)

    with ThreadPoolExecutor(workers()) as ex:
        res = list(ex.map(job, parts))
    out = {}
    for key in res[0]:
        if isinstance(res[0][key], list):
            out[key] = [v for r in res for v in r[key]]
        else:
            out[key] = np.concatenate([r[key] for r in res])
    return out


def oracle_requests(ora, xy, offs, agg):
    """Per-request tile, position and flag of the oracle's own pooled lists."""
    n = len(offs) - 1
    tile, pos, flags = np.zeros((n, 2), np.int64), np.zeros((n, 2)), np.zeros(n, np.int32)
    for r in range(n):
        ix, iy, x, y, fl = oracle.aggregate(ora["idx"][offs[r]:offs[r + 1]].ravel(), xy, *agg)
        tile[r], pos[r], flags[r] = (ix, iy), (x, y), fl
    ora.update(tile=tile, pos=pos, flags=flags)
    return ora


def sample_requests(offs, want_frames, seed):
    """Sorted random requests whose frames add up to at least want_frames."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(offs) - 1)
    chosen, total = [], 0
    for r in order:
        chosen.append(int(r))
        total += int(offs[r + 1] - offs[r])
        if total >= want_frames:
            break
    return np.sort(np.asarray(chosen))


def run_batch(torch, db, w, precision):
    q = torch.from_numpy(w.q).to("cuda:0")
    offs = torch.from_numpy(w.req_offsets.astype(np.int32)).to("cuda:0")
    t0 = time.perf_counter()
    out = db.query(q, w.k, w.n_reg, offs, precision=precision)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {key: v.cpu().numpy() for key, v in out.items()}
    res["regions"] = db.last_regions()
    res["info"] = db.info()
    say(f"[gpu] {w.name} {precision}: {len(w.q)} frames in {dt * 1e3:.1f} ms (first call), "
        f"info {res['info']}")
    return res


def judge_sample(w, res, reps, want_frames, seed):
    """Judges the frames of sampled whole requests and their estimates."""
    offs = np.asarray(w.req_offsets)
    reqs = sample_requests(offs, want_frames, seed)
    frames = np.concatenate([np.arange(offs[r], offs[r + 1]) for r in reqs])
    sub_offs = np.concatenate([[0], np.cumsum(offs[reqs + 1] - offs[reqs])])
    q = w.q[frames]
    t0 = time.perf_counter()
    ora = pooled_retrieve(w, q, w.k, reps)
    oracle_requests(ora, w.xy, sub_offs, w.agg)
    say(f"[oracle] {len(frames)} frames of {len(reqs)} requests in "
        f"{time.perf_counter() - t0:.1f} s on {workers()} threads")
    st = judge_frames(res["idx"][frames], res["dist"][frames], res["regions"][frames], ora,
                      w.feats, w.region_of, w.n_regions_total, q, w.k, reps=reps)
    same = judge_requests(res["idx"][frames], res["xy"][reqs], res["tile"][reqs],
                          res["flags"][reqs], ora, w.xy, sub_offs, w.agg)
    say(f"[ok] {w.name}: {st} same_pools={same}/{len(reqs)}")
    return st, same, len(reqs)


def assert_bitwise(a, b, what):
    for key in ("idx", "dist", "xy", "tile", "flags", "regions"):
        assert a[key].tobytes() == b[key].tobytes(), f"{what}: {key} differs"


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(hloc.LIB_PATH):
        pytest.fail("libhloc.so is not built")
    return torch


@pytest.fixture(scope="module")
def db_2m(torch_cuda):
    """The 2M x 512 database (bf16 and fp8 mirrors) with the precision
    shape's queries, and the oracle's region means."""
    t0 = time.perf_counter()
    say("[setup] drawing bf16-2m-d512 (2,000,000 x 512, 4,096 lognormal regions)")
    w = workload.make_workload(2)
    say(f"[setup] drawn in {time.perf_counter() - t0:.0f} s; building the device database")
    db = hloc.HlocDB(w.feats, w.xy, mirrors=ALL_MIRRORS)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    t1 = time.perf_counter()
    reps, _ = oracle.region_means(w.feats, w.region_of, w.n_regions_total)
    say(f"[setup] oracle region means in {time.perf_counter() - t1:.0f} s")
    yield w, db, reps
    db.close()


@pytest.fixture(scope="module")
def db_4m(torch_cuda):
    t0 = time.perf_counter()
    say("[setup] drawing serve-4m-d256 (4,000,000 x 256, 16,384 lognormal regions)")
    w = workload.make_workload(4)
    say(f"[setup] drawn in {time.perf_counter() - t0:.0f} s; building the device database")
    db = hloc.HlocDB(w.feats, w.xy, mirrors=ALL_MIRRORS)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    t1 = time.perf_counter()
    reps, _ = oracle.region_means(w.feats, w.region_of, w.n_regions_total)
    say(f"[setup] oracle region means in {time.perf_counter() - t1:.0f} s")
    yield w, db, reps
    db.close()


def test_full_precision_shape(torch_cuda, db_2m):
    """bf16-2m-d512: 2,048 single frames, n_regions 8, k 16; the bf16 screen
    (the chosen form) against the plain fp32 one and the oracle."""
    w, db, reps = db_2m
    say("[case] bf16-2m-d512 x2048, bf16 / fp32 / fp8 screens")
    res = run_batch(torch_cuda, db, w, "bf16")
    for prec in ("fp32", "fp8"):
        assert_bitwise(res, run_batch(torch_cuda, db, w, prec), f"bf16 vs {prec}")
    st, same, n = judge_sample(w, res, reps, SAMPLE_FRAMES, seed=2)
    assert st["frames"] >= SAMPLE_FRAMES
    assert st["recall"] >= 1.0 - st["tie_excused"] / st["frames"]


def test_full_multiframe_shape(torch_cuda, db_2m):
    """fp8-2m-d512-8frame: 4,096 requests of 8 frames (32,768 frames) on the
    same database, k 32, the paper's aggregation constants; fp8, bf16 and
    fp32 screens bit for bit, 128 whole requests against the oracle."""
    w2, db, reps = db_2m
    w = workload.make_workload(3, database=(w2.feats, w2.xy, w2.region_of))
    db.set_aggregation(*w.agg)
    say("[case] fp8-2m-d512-8frame 4096 x 8, fp8 / bf16 / fp32 screens")
    res = run_batch(torch_cuda, db, w, "fp8")
    for prec in ("bf16", "fp32"):
        assert_bitwise(res, run_batch(torch_cuda, db, w, prec), f"fp8 vs {prec}")
    st, same, n = judge_sample(w, res, reps, SAMPLE_FRAMES, seed=3)
    assert st["frames"] >= SAMPLE_FRAMES
    assert st["recall"] >= 1.0 - st["tie_excused"] / st["frames"]
    assert same >= n - st["tie_excused"] - st["region_excused"]


def test_full_exhaustive_shape(torch_cuda, db_2m):
    """bf16-2m-d512 searched exhaustively (n_regions = every region, the
    paper's whole-database search): 2,048 frames against all 2,000,000 rows,
    k 16; the bf16 screen against the plain fp32 one bit for bit, and sampled
    frames against the oracle's brute force over every row (12 frames: each
    costs the oracle tens of GB and seconds, so two at a time)."""
    w, db, reps = db_2m
    R = w.n_regions_total
    say(f"[case] bf16-2m-d512 x{len(w.q)} exhaustive (n_regions {R}), bf16 / fp32 screens")
    q = torch_cuda.from_numpy(w.q).to("cuda:0")
    offs = torch_cuda.from_numpy(w.req_offsets.astype(np.int32)).to("cuda:0")
    res = {}
    for prec in ("bf16", "fp32"):
        t0 = time.perf_counter()
        out = db.query(q, w.k, R, offs, precision=prec)
        torch_cuda.cuda.synchronize()
        res[prec] = {key: v.cpu().numpy() for key, v in out.items()}
        say(f"[gpu] exhaustive {prec}: {time.perf_counter() - t0:.2f} s (first call), "
            f"info {db.info()}")
    for key in ("idx", "dist", "xy", "tile", "flags"):
        assert res["bf16"][key].tobytes() == res["fp32"][key].tobytes(), f"exhaustive: {key}"
    frames = np.sort(np.random.default_rng(5).choice(len(w.q), 12, replace=False))
    t0 = time.perf_counter()

    def job(i):
        return oracle.retrieve(w.feats, w.region_of, R, w.q[i:i + 1], w.k, R, reps=reps)

    with ThreadPoolExecutor(2) as ex:
        parts = list(ex.map(job, frames.tolist()))
    ora = {key: (np.concatenate([p[key] for p in parts]) if not isinstance(parts[0][key], list)
                 else [v for p in parts for v in p[key]]) for key in parts[0]}
    say(f"[oracle] {len(frames)} frames by brute force in {time.perf_counter() - t0:.1f} s")
    st = judge_frames(res["bf16"]["idx"][frames], res["bf16"]["dist"][frames], None, ora,
                      w.feats, w.region_of, R, w.q[frames], w.k, reps=reps)
    say(f"[ok] bf16-2m-d512 exhaustive: {st}")
    assert st["frames"] == len(frames)
    assert st["recall"] >= 1.0 - st["tie_excused"] / st["frames"]


def test_full_serving_shape(torch_cuda, db_4m):
    """serve-4m-d256: 4,096 requests of 1-16 frames in one batch, k 32, on
    the 4M x 256 database; fp32, bf16 and fp8 screens bit for bit, whole
    requests of at least 1,024 frames against the oracle."""
    w, db, reps = db_4m
    say(f"[case] serve-4m-d256 {len(w.req_offsets) - 1} requests, {len(w.q)} frames")
    res = run_batch(torch_cuda, db, w, "bf16")
    for prec in ("fp32", "fp8"):
        assert_bitwise(res, run_batch(torch_cuda, db, w, prec), f"bf16 vs {prec}")
    st, same, n = judge_sample(w, res, reps, SAMPLE_FRAMES, seed=4)
    assert st["frames"] >= SAMPLE_FRAMES
    assert st["recall"] >= 1.0 - st["tie_excused"] / st["frames"]
    assert same >= n - st["tie_excused"] - st["region_excused"]


def test_full_serving_server(torch_cuda, db_4m):
    """The request server on the 4M x 256 database (bf16 screen): requests of
    1-16 frames with k in {8, 16, 32} from two threads; each result is the
    first k of the batch's k = 32 lists (one total order) and its estimate is
    the oracle's aggregation of exactly those candidates."""
    import threading
    w, db, reps = db_4m
    offs = np.asarray(w.req_offsets)
    rng = np.random.default_rng(44)
    reqs = [(int(r), int(rng.choice([8, 16, 32]))) for r in rng.choice(len(offs) - 1, 64,
                                                                       replace=False)]
    say(f"[case] server on serve-4m-d256: {len(reqs)} requests, bf16 screen")
    ref = run_batch(torch_cuda, db, w, "bf16")
    srv = hloc.Server(db, k=32, n_regions=w.n_reg, precision="bf16", max_batch_frames=256,
                      max_slots=3, max_queue_frames=8192)
    results = [None] * len(reqs)
    errors = []

    def client(ids):
        try:
            tickets = [(i, srv.submit(w.q[offs[reqs[i][0]]:offs[reqs[i][0] + 1]], reqs[i][1]))
                       for i in ids]
            for i, t in tickets:
                r, k = reqs[i]
                results[i] = srv.wait(t, int(offs[r + 1] - offs[r]), k)
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=client, args=(list(range(j, len(reqs), 2)),))
               for j in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    srv.close()
    assert not errors, errors
    for i, (r, k) in enumerate(reqs):
        got = results[i]
        fr = slice(offs[r], offs[r + 1])
        np.testing.assert_array_equal(got["idx"], ref["idx"][fr, :k])
        np.testing.assert_array_equal(got["dist"].view(np.uint32),
                                      ref["dist"][fr, :k].view(np.uint32))
        ix, iy, x, y, fl = oracle.aggregate(got["idx"].ravel(), w.xy, *w.agg)
        assert got["tile"].tolist() == [ix, iy] and got["flags"] == fl, f"request {r}"
        assert got["xy"].tolist() == [x, y] or (np.isnan(x) and np.isnan(got["xy"][0]))
    say(f"[ok] {len(reqs)} server requests equal the batch prefixes")
