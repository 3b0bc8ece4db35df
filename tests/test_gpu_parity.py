"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Each test builds a database on cuda:0, runs a batch through
hloc_query_batch[_async] and judges every frame and request with the
acceptance rule of tests/parity.py.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from parity import judge_frames, judge_requests
from paper_2006_08861_amd import hloc, workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MIRRORS = {"fp32": 0, "bf16": hloc.MIRROR_BF16, "fp8": hloc.MIRROR_FP8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(hloc.LIB_PATH):
        pytest.fail("libhloc.so is not built")
    return torch


def make_db(feats, xy, region_of, R, agg=None, reps=None, mirrors=0):
    db = hloc.HlocDB(feats, xy, mirrors=mirrors)
    db.set_regions(region_of, R, reps)
    if agg is not None:
        db.set_aggregation(*agg)
    return db


def run_device(torch, db, q, k, n_reg, offs=None, precision="fp32"):
    qd = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to("cuda:0")
    od = None if offs is None else torch.from_numpy(np.asarray(offs, np.int32)).to("cuda:0")
    out = db.query(qd, k, n_reg, od, precision=precision)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def check_all(torch, feats, xy, region_of, R, q, k, n_reg, offs=None, agg=(0.5, 1, 0.0, 0),
              reps=None, name="", precision="fp32"):
    say(f"[case] {name}: n={len(feats)} d={feats.shape[1]} R={R} nq={len(q)} k={k} "
        f"n_reg={n_reg} screen={precision}")
    db = make_db(feats, xy, region_of, R, agg, reps, mirrors=MIRRORS[precision])
    offs = np.arange(len(q) + 1) if offs is None else np.asarray(offs)
    out = run_device(torch, db, q, k, n_reg, offs, precision=precision)
    regs = db.last_regions()
    info = db.info()
    ora = oracle.localize(feats, xy, region_of, R, q, offs, k, n_reg, agg, reps=reps)
    st = judge_frames(out["idx"], out["dist"], regs, ora, feats, region_of, R, q, k, reps=reps)
    same = judge_requests(out["idx"], out["xy"], out["tile"], out["flags"], ora, xy, offs, agg)
    say(f"[ok] {name}: {st} same_pools={same}/{len(offs) - 1} info={info}")
    db.close()
    return st, info, out


# ------------------------------------------------------------- workload shapes
def test_cpu_shape_full_batch(torch_cuda):
    w = workload.make_workload(0)
    st, info, _ = check_all(torch_cuda, w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.k,
                            w.n_reg, w.req_offsets, w.agg, name="cpu-10k-d256 x1000")
    assert st["recall"] == 1.0


@pytest.fixture(scope="module")
def fp32_shape(torch_cuda):
    w = workload.make_workload(1)
    db = make_db(w.feats, w.xy, w.region_of, w.n_regions_total, w.agg)
    yield w, db
    db.close()


def test_fp32_shape_full_batch(torch_cuda, fp32_shape):
    w, db = fp32_shape
    say("[case] fp32-200k-d256 x256 (the benchmark's batch)")
    out = run_device(torch_cuda, db, w.q, w.k, w.n_reg, w.req_offsets)
    regs = db.last_regions()
    ora = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.req_offsets,
                          w.k, w.n_reg, w.agg)
    st = judge_frames(out["idx"], out["dist"], regs, ora, w.feats, w.region_of,
                      w.n_regions_total, w.q, w.k)
    same = judge_requests(out["idx"], out["xy"], out["tile"], out["flags"], ora, w.xy,
                          w.req_offsets, w.agg)
    say(f"[ok] {st} same_pools={same} info={db.info()}")
    assert st["recall"] == 1.0


def test_batch_invariance(torch_cuda, fp32_shape):
    # a frame's result must not depend on its batch-mates: bitwise equal alone,
    # in a subset, in reverse order and in the full batch
    w, db = fp32_shape
    say("[case] batch invariance on fp32-200k-d256")
    full = run_device(torch_cuda, db, w.q, w.k, w.n_reg)
    rng = np.random.default_rng(5)
    for sel in (np.arange(17), rng.choice(len(w.q), 40, replace=False), np.arange(len(w.q))[::-1],
                np.array([100])):
        part = run_device(torch_cuda, db, w.q[sel], w.k, w.n_reg)
        np.testing.assert_array_equal(part["idx"], full["idx"][sel])
        np.testing.assert_array_equal(part["dist"].view(np.uint32), full["dist"][sel].view(np.uint32))
        np.testing.assert_array_equal(part["xy"].view(np.uint64), full["xy"][sel].view(np.uint64))


def test_exhaustive_full_shape(torch_cuda, fp32_shape):
    """n_regions = R on fp32-200k-d256: every frame against all 200,000 rows
    (all items wide), 48 frames checked against the oracle's exhaustive
    search, and bitwise the same lists alone as in the batch."""
    w, db = fp32_shape
    R = w.n_regions_total
    say("[case] exhaustive fp32-200k-d256 x48")
    q = w.q[:48]
    out = run_device(torch_cuda, db, q, w.k, R)
    regs = db.last_regions()
    ora = oracle.localize(w.feats, w.xy, w.region_of, R, q, np.arange(len(q) + 1), w.k, R,
                          w.agg)
    st = judge_frames(out["idx"], out["dist"], regs, ora, w.feats, w.region_of, R, q, w.k)
    say(f"[ok] {st} info={db.info()}")
    assert st["recall"] == 1.0
    one = run_device(torch_cuda, db, q[7:8], w.k, R)
    np.testing.assert_array_equal(one["idx"][0], out["idx"][7])
    np.testing.assert_array_equal(one["dist"][0].view(np.uint32), out["dist"][7].view(np.uint32))


def test_sliding_windows(torch_cuda):
    """Windows of M = 11 frames (Section 4's window) over a 120-frame video
    along the walk, each frame retrieved once (hloc_query_windows_async):
    frame lists against the oracle, every request against the oracle's
    estimate, and bitwise against the same windows sent as materialised
    requests; a list naming a frame outside the batch flags only its request."""
    torch = torch_cuda
    w = workload.make_workload(0, nq=8)
    rng = np.random.default_rng(21)
    T, M = 120, 11
    q = (w.feats[3000:3000 + T] + 0.1 * rng.standard_normal((T, w.feats.shape[1]))
         ).astype(np.float32)
    starts = np.arange(T - M + 1)
    frames = np.concatenate([np.arange(s0, s0 + M) for s0 in starts]).astype(np.int32)
    offs = (np.arange(len(starts) + 1) * M).astype(np.int32)
    agg = (0.3, 10, 3.0, 20)
    say(f"[case] sliding windows T={T} M={M}")
    db = make_db(w.feats, w.xy, w.region_of, w.n_regions_total, agg)
    out = db.query_windows(q, w.k, w.n_reg, offs, frames)
    torch.cuda.synchronize()
    out = {key: v.cpu().numpy() for key, v in out.items()}
    regs = db.last_regions()
    ora = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, q, offs, w.k, w.n_reg,
                          agg, req_frames=frames)
    st = judge_frames(out["idx"], out["dist"], regs, ora, w.feats, w.region_of,
                      w.n_regions_total, q, w.k)
    assert st["recall"] == 1.0
    same_frames = np.array([set(out["idx"][i].tolist()) == set(ora["idx"][i].tolist())
                            for i in range(T)])
    checked = 0
    for r in range(len(starts)):
        fr = frames[offs[r]:offs[r + 1]]
        if not same_frames[fr].all():
            continue
        checked += 1
        assert out["tile"][r].tolist() == ora["tile"][r].tolist(), r
        assert out["flags"][r] == ora["flags"][r], r
        assert out["xy"][r].tolist() == ((ora["tile"][r] + 0.5) * agg[0]).tolist(), r
    say(f"[ok] {st} windows checked {checked}/{len(starts)}")
    assert checked >= len(starts) - 5
    mat = run_device(torch, db, q[frames], w.k, w.n_reg, offs)
    for key in ("tile", "flags"):
        np.testing.assert_array_equal(mat[key], out[key])
    np.testing.assert_array_equal(mat["xy"].view(np.uint64), out["xy"].view(np.uint64))
    bad = frames.copy()
    bad[2 * M + 3] = T + 5
    out2 = db.query_windows(q, w.k, w.n_reg, offs, bad)
    torch.cuda.synchronize()
    flags2 = out2["flags"].cpu().numpy()
    assert flags2[2] == hloc.FLAG_BAD_REQUEST
    np.testing.assert_array_equal(np.delete(flags2, 2), np.delete(out["flags"], 2))
    db.close()


def test_streams_across_calls(torch_cuda):
    """Sliding windows of M = 11 across calls (hloc_streams): two video
    streams of 60 frames sent in three calls of uneven pieces, each frame
    once. Every frame's list against the oracle, every window's estimate
    against the oracle's for that window (the frame and up to 10 before it in
    its stream) and bit for bit against the same windows sent in one batch as
    materialised requests. A stream repeated in a call and an out-of-range
    stream are flagged and leave the history as it was; a reset empties it."""
    torch = torch_cuda
    w = workload.make_workload(0, nq=8)
    rng = np.random.default_rng(23)
    T, M, S = 60, 11, 2
    d = w.feats.shape[1]
    videos = [(w.feats[3000 + 2500 * s:3000 + 2500 * s + T + 1]
               + 0.1 * rng.standard_normal((T + 1, d))).astype(np.float32) for s in range(S)]
    agg = (0.3, 10, 3.0, 20)
    R = w.n_regions_total
    say(f"[case] streams across calls: {S} videos x {T} frames, M={M}")
    db = make_db(w.feats, w.xy, w.region_of, R, agg)
    st = hloc.Streams(db, n_streams=4, window=M, k=w.k, max_frames=64)

    def send(call):
        q = np.concatenate([videos[s][a:b] for s, a, b in call])
        offs = np.cumsum([0] + [b - a for s, a, b in call]).astype(np.int32)
        sid = np.array([s for s, a, b in call], np.int32)
        out = st.query(q, offs, sid, w.n_reg)
        torch.cuda.synchronize()
        return {key: v.cpu().numpy() for key, v in out.items()}

    got = {}
    for call in ([(0, 0, 25), (1, 0, 7)], [(1, 7, 41), (0, 25, 30)], [(0, 30, 60), (1, 41, 60)]):
        out = send(call)
        j = 0
        for s, a, b in call:
            for t in range(a, b):
                got[(s, t)] = {key: out[key][j] for key in out}
                j += 1
    allq = np.concatenate([v[:T] for v in videos])  # frame (s, t) at s T + t
    frames, offs = [], [0]
    for s in range(S):
        for t in range(T):
            frames += [s * T + u for u in range(max(0, t - M + 1), t + 1)]
            offs.append(len(frames))
    frames, offs = np.asarray(frames, np.int32), np.asarray(offs, np.int32)
    ora = oracle.localize(w.feats, w.xy, w.region_of, R, allq, offs, w.k, w.n_reg, agg,
                          req_frames=frames)
    keys = [(s, t) for s in range(S) for t in range(T)]
    idx = np.stack([got[kk]["idx"] for kk in keys])
    dist = np.stack([got[kk]["dist"] for kk in keys])
    st_ = judge_frames(idx, dist, None, ora, w.feats, w.region_of, R, allq, w.k)
    assert st_["recall"] == 1.0
    same = np.array([set(idx[i].tolist()) == set(ora["idx"][i].tolist()) for i in range(len(keys))])
    checked = 0
    for r, kk in enumerate(keys):
        if not same[frames[offs[r]:offs[r + 1]]].all():
            continue
        checked += 1
        assert got[kk]["tile"].tolist() == ora["tile"][r].tolist(), kk
        assert got[kk]["flags"] == ora["flags"][r], kk
    say(f"[ok] {st_} windows checked {checked}/{len(keys)}")
    assert checked >= len(keys) - 5
    mat = run_device(torch, db, allq[frames], w.k, w.n_reg, offs)
    for r, kk in enumerate(keys):
        assert mat["tile"][r].tolist() == got[kk]["tile"].tolist(), kk
        assert mat["flags"][r] == got[kk]["flags"], kk
        assert mat["xy"][r].tobytes() == got[kk]["xy"].tobytes(), kk
    # a repeated stream and an out-of-range one: flagged, histories unchanged
    bad = send([(0, T, T + 1), (0, T, T + 1), (3, 0, 1)][:2])
    assert (bad["flags"] == hloc.FLAG_BAD_REQUEST).all()
    q_bad = np.concatenate([videos[0][T:T + 1]])
    out = st.query(q_bad, np.array([0, 1], np.int32), np.array([7], np.int32), w.n_reg)
    torch.cuda.synchronize()
    assert out["flags"].cpu().numpy()[0] == hloc.FLAG_BAD_REQUEST
    # frame T of stream 0: its window is frames T - 10 .. T of video 0
    last = send([(0, T, T + 1)])
    q_last = np.concatenate([videos[0][T - M + 1:T + 1]])
    ref = run_device(torch, db, q_last, w.k, w.n_reg, np.array([0, M], np.int32))
    assert last["tile"][0].tolist() == ref["tile"][0].tolist()
    assert last["xy"][0].tobytes() == ref["xy"][0].tobytes()
    assert last["flags"][0] == ref["flags"][0]
    # after a reset a frame's window is the frame alone
    st.reset()
    one = send([(1, 5, 6)])
    ref1 = run_device(torch, db, videos[1][5:6], w.k, w.n_reg, np.array([0, 1], np.int32))
    assert one["xy"][0].tobytes() == ref1["xy"][0].tobytes()
    st.close()
    db.close()


@pytest.mark.parametrize("n_reg", [5, 1000])
def test_subspace_labels(torch_cuda, n_reg):
    """Top k per (frame, label) over three labels (contiguous runs of regions,
    like walked paths) and requests of 5 frames pooling frames x labels x k:
    every (label, frame) list judged against the oracle's label-restricted
    search with the acceptance rule (tie band, region ties re-judged on the
    GPU's regions), every request's estimate bit for bit against the oracle's
    aggregation of the GPU's pooled candidates; n_regions = 1000 searches
    every region of each label. A label count other than the one set is
    refused; one label covering all regions gives the plain query bitwise."""
    torch = torch_cuda
    w = workload.make_workload(0, nq=60)
    R = w.n_regions_total
    P = 3
    labels = ((np.arange(R) * P) // R).astype(np.int32)
    offs = np.arange(0, 61, 5).astype(np.int32)
    agg = (0.3, 10, 3.0, 20)
    say(f"[case] labels P={P} n_reg={n_reg}")
    db = make_db(w.feats, w.xy, w.region_of, R, agg)
    db.set_region_labels(labels, P)
    with pytest.raises(hloc.HlocError) as e:
        db.query_labels(w.q, w.k, n_reg, P - 1, offs)
    assert e.value.code == hloc.EINVAL
    out = db.query_labels(w.q, w.k, n_reg, P, offs)
    torch.cuda.synchronize()
    out = {key: v.cpu().numpy() for key, v in out.items()}
    nq = len(w.q)
    sizes = np.bincount(w.region_of, minlength=R)
    per_label = np.bincount(labels[sizes > 0], minlength=P)
    # with n_regions within every label's regions the labels run as one batch
    # (frame p * nq + f under label p) and the device's region choice is kept
    one_batch = n_reg <= per_label.min()
    regs = db.last_regions() if one_batch else None
    ora = oracle.localize_labels(w.feats, w.xy, w.region_of, R, labels, w.q, offs, w.k, n_reg,
                                 agg)
    for p in range(P):
        gr = regs[p * nq:(p + 1) * nq] if one_batch else None
        if not one_batch:
            # every region of the label is searched: no choice to compare
            assert all(len(r) == per_label[p] for r in ora["per_label"][p]["regions"])
        st = judge_frames(out["idx"][p], out["dist"][p], gr, ora["per_label"][p], w.feats,
                          w.region_of, R, w.q, w.k)
        say(f"[ok] label {p}: {st}")
        got = out["idx"][p][out["idx"][p] >= 0]
        assert np.all(labels[w.region_of[got]] == p)
    same = 0
    for r in range(len(offs) - 1):
        pooled = out["idx"][:, offs[r]:offs[r + 1]].transpose(1, 0, 2).ravel()
        ix, iy, x, y, fl = oracle.aggregate(pooled, w.xy, *agg)
        assert out["tile"][r].tolist() == [ix, iy] and int(out["flags"][r]) == fl, r
        assert out["xy"][r].tolist() == [x, y], r
        o_pooled = ora["idx"][:, offs[r]:offs[r + 1]].transpose(1, 0, 2).ravel()
        if sorted(pooled.tolist()) == sorted(o_pooled.tolist()):
            same += 1
            assert out["tile"][r].tolist() == ora["tile"][r].tolist(), r
            assert out["flags"][r] == ora["flags"][r], r
    say(f"[ok] requests with the oracle's pooled candidates: {same}/{len(offs) - 1}")
    db.set_region_labels(np.zeros(R, np.int32), 1)
    one = db.query_labels(w.q, w.k, n_reg, 1, offs)
    plain = run_device(torch, db, w.q, w.k, n_reg, offs)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(one["idx"][0].cpu().numpy(), plain["idx"])
    np.testing.assert_array_equal(one["tile"].cpu().numpy(), plain["tile"])
    db.close()


def test_host_and_device_entry_points_agree(torch_cuda, fp32_shape):
    w, db = fp32_shape
    say("[case] sync host-pointer call vs async device call")
    dev = run_device(torch_cuda, db, w.q[:64], w.k, w.n_reg)
    host = db.query(w.q[:64], w.k, w.n_reg)
    for key in ("idx", "dist", "tile", "flags"):
        np.testing.assert_array_equal(host[key], dev[key])
    np.testing.assert_array_equal(host["xy"].view(np.uint64), dev["xy"].view(np.uint64))


def test_multiframe_paper_aggregation(torch_cuda):
    w = workload.make_workload(3, nq=48, n=20_000)
    st, info, _ = check_all(torch_cuda, w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.k,
                            w.n_reg, w.req_offsets, w.agg, name="8-frame requests, d512")
    assert st["recall"] == 1.0


def test_serving_shape_mixed_frames(torch_cuda):
    w = workload.make_workload(4, nq=40, n=30_000)
    st, info, _ = check_all(torch_cuda, w.feats, w.xy, w.region_of, w.n_regions_total, w.q, 16,
                            w.n_reg, w.req_offsets, w.agg, name="1-16 frame requests, d256")
    assert st["recall"] == 1.0


# ------------------------------------------------------------- edge cases
def _random_db(seed, n, d, R, empty=0, dist="normal"):
    rng = np.random.default_rng(seed)
    feats = rng.standard_normal((n, d)).astype(np.float32)
    region_of = rng.integers(0, R - empty, size=n).astype(np.int32)
    if empty:
        # move some ids to the top so that ids R-empty..R-1 are empty; shuffle ids
        perm = rng.permutation(R)
        region_of = perm[region_of].astype(np.int32)
    xy = rng.uniform(0, 60, size=(n, 2))
    return rng, feats, xy, region_of


def test_ragged_dims_empty_regions(torch_cuda):
    rng, feats, xy, region_of = _random_db(1, 1500, 37, 40, empty=6)
    q = (feats[rng.integers(0, 1500, 45)] + 0.3 * rng.standard_normal((45, 37))).astype(np.float32)
    for k, n_reg in ((7, 3), (1, 1), (33, 5)):
        st, _, _ = check_all(torch_cuda, feats, xy, region_of, 40, q, k, n_reg,
                             name=f"d37 empty regions k{k}")
        assert st["recall"] == 1.0


@pytest.mark.parametrize("nq,n_reg", [(1500, 4), (600, 12), (300, 8), (1200, 8)])
def test_schedule_paths(torch_cuda, nq, n_reg):
    # the one-block schedule keeps a frame's regions in registers when every
    # frame has its own thread and keeps at most 8 regions; more frames than
    # threads, or more regions per frame, take its general loop; more than
    # 8,192 (frame, region) pairs over few regions take the multi-kernel
    # schedule with per-block LDS counts
    rng, feats, xy, region_of = _random_db(4, 4000, 48, 120, empty=5)
    q = (feats[rng.integers(0, 4000, nq)] + 0.2 * rng.standard_normal((nq, 48))).astype(np.float32)
    st, _, _ = check_all(torch_cuda, feats, xy, region_of, 120, q, 9, n_reg,
                         name=f"schedule nq={nq} n_regions={n_reg}")
    assert st["recall"] == 1.0


@pytest.mark.parametrize("many", [False, True])
def test_requests_with_large_pools(torch_cuda, many):
    # requests pooling more than 512 candidates: with at most one request per
    # compute unit one launch takes every request; with more, they are listed
    # for the large-list kernel and the others take the small one
    rng, feats, xy, region_of = _random_db(5, 5000, 32, 50)
    if many:
        sizes = [16 if r % 50 == 0 else 1 for r in range(300)] + [24]
    else:
        sizes = [16, 1, 16, 7, 24]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    nq = int(offs[-1])
    q = (feats[rng.integers(0, 5000, nq)] + 0.2 * rng.standard_normal((nq, 32))).astype(np.float32)
    st, _, out = check_all(torch_cuda, feats, xy, region_of, 50, q, 40, 5, offs,
                           agg=(0.5, 3, 1.0, 20),
                           name=f"pools of 40 to 960 candidates, {len(sizes)} requests")
    assert st["recall"] == 1.0
    assert np.all(out["flags"] & 6 == 0)  # neither empty nor rejected


def test_exhaustive_mode(torch_cuda):
    rng, feats, xy, region_of = _random_db(2, 2000, 24, 20)
    q = rng.standard_normal((33, 24)).astype(np.float32)
    for n_reg in (20, 1000):
        st, _, out = check_all(torch_cuda, feats, xy, region_of, 20, q, 12, n_reg,
                               name=f"exhaustive n_regions={n_reg}")
        assert st["recall"] == 1.0


def test_padding_when_candidates_run_out(torch_cuda):
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 4, size=30)
    region_of = np.repeat(np.arange(30), sizes).astype(np.int32)
    n = len(region_of)
    feats = rng.standard_normal((n, 16)).astype(np.float32)
    xy = rng.uniform(0, 10, size=(n, 2))
    q = rng.standard_normal((20, 16)).astype(np.float32)
    st, _, out = check_all(torch_cuda, feats, xy, region_of, 30, q, 8, 1, name="padding")
    assert (out["idx"] == -1).any() and np.isinf(out["dist"]).any()


def test_exact_match_queries(torch_cuda):
    rng, feats, xy, region_of = _random_db(4, 3000, 64, 30)
    js = rng.integers(0, 3000, 64)
    st, _, out = check_all(torch_cuda, feats, xy, region_of, 30, feats[js], 5, 30,
                           name="exact match")
    assert (out["idx"][:, 0] == js).all() and (out["dist"][:, 0] == 0).all()


def test_duplicate_rows_break_ties_by_index_and_fall_back(torch_cuda):
    # 200 identical rows: the screen cannot separate them, so the certificate
    # fails and the exact FP64 pass decides; ties go to the smaller index
    rng = np.random.default_rng(6)
    n, d = 1200, 32
    feats = rng.standard_normal((n, d)).astype(np.float32)
    dup = rng.choice(n, 200, replace=False)
    feats[dup] = feats[dup[0]]
    region_of = (np.arange(n) % 7).astype(np.int32)
    xy = rng.uniform(0, 20, size=(n, 2))
    q = np.repeat(feats[dup[:1]], 3, axis=0)
    st, info, out = check_all(torch_cuda, feats, xy, region_of, 7, q, 10, 7, name="duplicates")
    assert out["idx"][0].tolist() == sorted(dup.tolist())[:10]
    assert info["fine_fallbacks"] == 3
    # 1,500 identical rows: the uncertain band exceeds the re-score capacity
    # and every candidate of the frame is recomputed in FP64
    feats2 = rng.standard_normal((2400, d)).astype(np.float32)
    dup2 = rng.choice(2400, 1500, replace=False)
    feats2[dup2] = feats2[dup2[0]]
    region2 = (np.arange(2400) % 5).astype(np.int32)
    xy2 = rng.uniform(0, 20, size=(2400, 2))
    st, info, out = check_all(torch_cuda, feats2, xy2, region2, 5, feats2[dup2[:2]], 10, 5,
                              name="duplicates beyond the band capacity")
    assert out["idx"][0].tolist() == sorted(dup2.tolist())[:10]
    assert info["fine_fallbacks"] == 2


def test_identical_representatives_fall_back(torch_cuda):
    # sixteen regions holding the same rows have identical means, more than
    # the coarse shortlist (n_regions + 4) can hold: the coarse certificate
    # fails and the exact pass keeps the lowest region ids
    rng = np.random.default_rng(7)
    base = rng.standard_normal((50, 16)).astype(np.float32)
    other = rng.standard_normal((100, 16)).astype(np.float32) + 3.0
    feats = np.concatenate([np.tile(base, (16, 1)), other])
    region_of = np.concatenate([np.repeat(np.arange(16), 50),
                                16 + np.arange(100) % 12]).astype(np.int32)
    xy = rng.uniform(0, 20, size=(len(feats), 2))
    q = (base[:5] + 0.01).astype(np.float32)
    for precision in ("fp32", "bf16"):
        st, info, _ = check_all(torch_cuda, feats, xy, region_of, 28, q, 6, 3,
                                name=f"equal means, {precision} screens", precision=precision)
        assert info["coarse_fallbacks"] == 5


@pytest.mark.parametrize("n_same", [16, 120])
def test_fused_coarse_equal_means(torch_cuda, n_same):
    """The fused bf16 coarse product keeps, per frame and lane group, the 6
    best quads (representatives 4 q .. 4 q + 3), lane group g seeing the
    quads 4 g .. 4 g + 3 of every 16 representatives. n_same regions (ids
    0 .. n_same - 1) hold the same rows, so their means tie for the best.
    With 16 (one tied quad per group) the band of the kept keys settles the
    tie (coarse fallback); with 120 (7 or 8 tied quads per group, more than
    it keeps) the keys cannot decide and the frame is deferred to the dense
    coarse screen. Either way the lowest ids win, as in the fp32 path
    (bitwise) and the oracle."""
    rng = np.random.default_rng(11)
    d, rows = 64, 30
    base = rng.standard_normal((rows, d)).astype(np.float32)
    other = (rng.standard_normal((60 * 20, d)) + 2.0).astype(np.float32)
    feats = np.concatenate([np.tile(base, (n_same, 1)), other])
    region_of = np.concatenate([np.repeat(np.arange(n_same), rows),
                                n_same + np.arange(60 * 20) // 20]).astype(np.int32)
    R = n_same + 60
    xy = rng.uniform(0, 20, size=(len(feats), 2))
    q = (base[:5] + 0.01).astype(np.float32)
    outs = {}
    for precision in ("fp32", "bf16"):
        st, info, out = check_all(torch_cuda, feats, xy, region_of, R, q, 6, 3,
                                  name=f"{n_same} equal means, {precision} screens",
                                  precision=precision)
        outs[precision] = out
        assert st["recall"] == 1.0
        if precision == "bf16":
            if n_same == 16:
                assert info["coarse_fallbacks"] == 5 and info["coarse_deferred"] == 0
            else:
                assert info["coarse_deferred"] == 5
    for key in ("idx", "dist", "tile", "flags", "xy"):
        assert outs["fp32"][key].tobytes() == outs["bf16"][key].tobytes(), key


@pytest.mark.parametrize("n_reg", [5, 1000])
def test_subspace_labels_bf16(torch_cuda, n_reg):
    """Label queries through the bf16 screens (the fused coarse product then
    masks the regions of other labels itself): bitwise the fp32 screens'
    results, which test_subspace_labels judges against the oracle."""
    torch = torch_cuda
    w = workload.make_workload(0, nq=60)
    R = w.n_regions_total
    P = 3
    labels = ((np.arange(R) * P) // R).astype(np.int32)
    offs = np.arange(0, 61, 5).astype(np.int32)
    agg = (0.3, 10, 3.0, 20)
    say(f"[case] labels P={P} n_reg={n_reg}, bf16 vs fp32 screens")
    db = make_db(w.feats, w.xy, w.region_of, R, agg, mirrors=hloc.MIRROR_BF16)
    db.set_region_labels(labels, P)
    res = {}
    for precision in ("fp32", "bf16"):
        out = db.query_labels(w.q, w.k, n_reg, P, offs, precision=precision)
        torch.cuda.synchronize()
        res[precision] = {key: v.cpu().numpy() for key, v in out.items()}
    say(f"[ok] info {db.info()}")
    for key in ("idx", "dist", "tile", "flags", "xy"):
        assert res["fp32"][key].tobytes() == res["bf16"][key].tobytes(), key
    got = res["bf16"]["idx"]
    for p in range(P):
        g = got[p][got[p] >= 0]
        assert np.all(labels[w.region_of[g]] == p)
    db.close()


def test_user_representatives_and_relayout(torch_cuda):
    rng, feats, xy, region_of = _random_db(8, 2500, 48, 25)
    reps = rng.standard_normal((25, 48)).astype(np.float32)
    q = rng.standard_normal((30, 48)).astype(np.float32)
    st, _, _ = check_all(torch_cuda, feats, xy, region_of, 25, q, 9, 4, reps=reps,
                         name="given representatives")
    assert st["recall"] == 1.0
    # set regions twice on one database: the second layout starts from a permuted one
    say("[case] set_regions twice")
    db = make_db(feats, xy, region_of, 25)
    region2 = rng.integers(0, 11, size=2500).astype(np.int32)
    db.set_regions(region2, 11)
    out = run_device(torch_cuda, db, q, 9, 3)
    ora = oracle.retrieve(feats, region2, 11, q, 9, 3)
    st = judge_frames(out["idx"], out["dist"], db.last_regions(), ora, feats, region2, 11, q, 9)
    assert st["recall"] == 1.0
    db.close()


def test_max_dim_and_max_k(torch_cuda):
    rng, feats, xy, region_of = _random_db(9, 1800, 1024, 12)
    q = rng.standard_normal((20, 1024)).astype(np.float32)
    st, _, _ = check_all(torch_cuda, feats, xy, region_of, 12, q, 256, 6, name="d1024 k256")
    assert st["recall"] == 1.0


def test_empty_batch_and_bad_offsets(torch_cuda):
    import torch
    rng, feats, xy, region_of = _random_db(10, 500, 16, 5)
    say("[case] empty batch, bad offsets")
    db = make_db(feats, xy, region_of, 5)
    out = db.query(np.zeros((0, 16), np.float32), 4, 2)
    assert out["idx"].shape == (0, 4)
    q = rng.standard_normal((6, 16)).astype(np.float32)
    with pytest.raises(hloc.HlocError) as e:
        db.query(q, 4, 2, req_offsets=[0, 4, 2, 6])
    assert e.value.code == hloc.EINVAL
    # the device entry point cannot check offsets on the host: the request is flagged
    res = run_device(torch, db, q, 4, 2, offs=[0, 4, 2, 6])
    assert res["flags"].tolist()[1] == hloc.FLAG_BAD_REQUEST
    assert res["flags"].tolist()[0] in (0, hloc.FLAG_LOW_CONFIDENCE)
    with pytest.raises(hloc.HlocError) as e:
        db.query(q, 4, 2, precision="bf16")
    assert e.value.code == hloc.EUNSUPPORTED
    with pytest.raises(hloc.HlocError) as e:
        db.query(q, 0, 2)
    assert e.value.code == hloc.EINVAL
    db.close()


# ------------------------------------------------------------- aggregation
def _golden_cases():
    with open(os.path.join(GOLDEN, "aggregation_cases.json")) as f:
        return [c for c in json.load(f)["cases"] if -1 not in c.get("rows", [])]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_aggregation_golden_on_device(torch_cuda, case):
    # one database row per point; each frame is a copy of one row, searched
    # exhaustively with k = 1, so the pooled candidates are exactly the
    # case's rows and the device aggregation must give the hand-worked tile
    cell = case["cell"]
    if "tiles" in case:
        pts, rows = [], []
        for ix, iy, c in case["tiles"]:
            rows += [len(pts)] * c
            pts.append([(ix + 0.5) * cell, (iy + 0.5) * cell])
    else:
        pts, rows = case["points"], case.get("rows", list(range(len(case["points"]))))
    pts = np.asarray(pts, np.float64)
    n = len(pts)
    rng = np.random.default_rng(11)
    feats = rng.standard_normal((n, 32)).astype(np.float32)
    db = make_db(feats, pts, np.zeros(n, np.int32), 1,
                 (cell, case["top_c"], case["radius"], case["toler_pct"]))
    q = feats[np.asarray(rows)]
    out = run_device(torch_cuda, db, q, 1, 1, offs=[0, len(rows)])
    assert out["idx"][:, 0].tolist() == list(rows)
    assert out["tile"][0].tolist() == case["expect"]["tile"]
    assert int(out["flags"][0]) == case["expect"]["flag"]
    ix, iy = case["expect"]["tile"]
    assert out["xy"][0].tolist() == [(ix + 0.5) * cell, (iy + 0.5) * cell]
    db.close()


# ------------------------------------------------------------- workspaces, graphs
def _bitwise_equal(a, b):
    for key in ("idx", "dist", "tile", "flags", "xy"):
        x, y = a[key], b[key]
        if hasattr(x, "cpu"):
            x = x.cpu().numpy()
        if hasattr(y, "cpu"):
            y = y.cpu().numpy()
        assert x.shape == y.shape, key
        assert x.tobytes() == y.tobytes(), key


def test_graph_replay_matches_eager(torch_cuda, fp32_shape):
    # one captured batch replayed on changing inputs, with eager batches and
    # synchronizations between the replays; every replay equals the eager run
    torch = torch_cuda
    w, db = fp32_shape
    say("[case] captured batch replayed 4 times")
    ws = hloc.Workspace(db)
    nq = 96
    q_buf = torch.from_numpy(w.q[:nq]).cuda()
    out = hloc.Workspace.outputs(nq, nq, w.k, q_buf.device)
    ws.capture(q_buf, w.k, w.n_reg, None, out)
    s = torch.cuda.Stream()
    rng = np.random.default_rng(21)
    for rep in range(4):
        sel = rng.choice(len(w.q), nq, replace=False)
        q_buf.copy_(torch.from_numpy(w.q[sel]).cuda())
        torch.cuda.synchronize()
        ws.replay(s)
        s.synchronize()
        got = {k: v.clone() for k, v in out.items()}
        eager = run_device(torch, db, w.q[sel], w.k, w.n_reg)
        _bitwise_equal(got, eager)
    ws.close()


def test_graph_replay_refused_after_changes(torch_cuda, fp32_shape):
    """A captured graph holds buffer and database addresses: growing the
    workspace, or changing the database's regions or aggregation, makes a
    replay return ESTATE until the batch is captured again."""
    torch = torch_cuda
    w, _ = fp32_shape
    say("[case] graph invalidation")
    db = make_db(w.feats, w.xy, w.region_of, w.n_regions_total, w.agg)
    ws = hloc.Workspace(db)
    nq = 32
    q_buf = torch.from_numpy(w.q[:nq]).cuda()
    out = hloc.Workspace.outputs(nq, nq, w.k, q_buf.device)
    s = torch.cuda.Stream()
    ws.capture(q_buf, w.k, w.n_reg, None, out)
    ws.replay(s)
    s.synchronize()
    # a larger batch on the same workspace reallocates its buffers
    big = torch.from_numpy(w.q).cuda()
    big_out = hloc.Workspace.outputs(len(w.q), len(w.q), w.k, big.device)
    ws.query_async(big, w.k, w.n_reg, None, big_out, s)
    s.synchronize()
    with pytest.raises(hloc.HlocError) as e:
        ws.replay(s)
    assert e.value.code == hloc.ESTATE
    ws.capture(q_buf, w.k, w.n_reg, None, out)
    ws.replay(s)
    s.synchronize()
    _bitwise_equal(out, run_device(torch, db, w.q[:nq], w.k, w.n_reg))
    db.set_aggregation(*w.agg)
    with pytest.raises(hloc.HlocError) as e:
        ws.replay(s)
    assert e.value.code == hloc.ESTATE
    ws.capture(q_buf, w.k, w.n_reg, None, out)
    db.set_regions(w.region_of, w.n_regions_total)
    with pytest.raises(hloc.HlocError) as e:
        ws.replay(s)
    assert e.value.code == hloc.ESTATE
    ws.close()
    db.close()


def test_concurrent_workspaces_match_alone(torch_cuda, fp32_shape):
    # two batches in flight on two workspaces and two streams give the same
    # bits as each batch run alone
    torch = torch_cuda
    w, db = fp32_shape
    say("[case] two workspaces on two streams")
    qa = torch.from_numpy(w.q[:128]).cuda()
    qb = torch.from_numpy(w.q[128:]).cuda()
    wa, wb = hloc.Workspace(db), hloc.Workspace(db)
    oa = hloc.Workspace.outputs(128, 128, w.k, qa.device)
    ob = hloc.Workspace.outputs(128, 128, w.k, qa.device)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        wa.query_async(qa, w.k, w.n_reg, None, oa, sa)
        wb.query_async(qb, w.k, w.n_reg, None, ob, sb)
    torch.cuda.synchronize()
    _bitwise_equal(oa, run_device(torch, db, w.q[:128], w.k, w.n_reg))
    _bitwise_equal(ob, run_device(torch, db, w.q[128:], w.k, w.n_reg))
    wa.close()
    wb.close()


# ------------------------------------------------------------- bf16 screen
@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_lp_screen_fp32_shape(torch_cuda, precision):
    w = workload.make_workload(1)
    st, info, _ = check_all(torch_cuda, w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.k,
                            w.n_reg, w.req_offsets, w.agg, name="fp32-200k-d256",
                            precision=precision)
    assert st["recall"] == 1.0


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_lp_screen_multiframe_d512(torch_cuda, precision):
    w = workload.make_workload(3, nq=48, n=20_000)
    st, info, _ = check_all(torch_cuda, w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.k,
                            w.n_reg, w.req_offsets, w.agg, name="8-frame d512",
                            precision=precision)
    assert st["recall"] == 1.0


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_lp_screen_ragged_and_duplicates(torch_cuda, precision):
    rng, feats, xy, region_of = _random_db(31, 1500, 37, 40, empty=6)
    q = (feats[rng.integers(0, 1500, 45)] + 0.3 * rng.standard_normal((45, 37))).astype(np.float32)
    st, _, _ = check_all(torch_cuda, feats, xy, region_of, 40, q, 7, 3, name="d37",
                         precision=precision)
    assert st["recall"] == 1.0
    dup = rng.choice(1500, 300, replace=False)
    feats[dup] = feats[dup[0]]
    st, info, out = check_all(torch_cuda, feats, xy, region_of, 40, feats[dup[:2]], 10, 40,
                              name="duplicates", precision=precision)
    assert out["idx"][0].tolist() == sorted(dup.tolist())[:10]


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_lp_and_fp32_screens_agree_bitwise(torch_cuda, precision):
    # every screen ends in the same certified FP64 rerank: identical results
    torch = torch_cuda
    w = workload.make_workload(1, nq=128)
    say(f"[case] {precision} vs fp32 screen on one database")
    db = make_db(w.feats, w.xy, w.region_of, w.n_regions_total, w.agg, mirrors=MIRRORS[precision])
    a = run_device(torch, db, w.q, w.k, w.n_reg, precision="fp32")
    regs_a = db.last_regions()
    b = run_device(torch, db, w.q, w.k, w.n_reg, precision=precision)
    regs_b = db.last_regions()
    say(f"[ok] {precision} info {db.info()}")
    np.testing.assert_array_equal(regs_a, regs_b)  # the low-precision coarse stage agrees
    for key in ("idx", "dist", "tile", "flags", "xy"):
        assert a[key].tobytes() == b[key].tobytes(), key
    db.close()


def test_fp8_needs_a_multiple_of_64(torch_cuda):
    rng, feats, xy, region_of = _random_db(32, 300, 20, 6)  # padded length 32
    db = make_db(feats, xy, region_of, 6, mirrors=hloc.MIRROR_FP8)
    with pytest.raises(hloc.HlocError) as e:
        run_device(torch_cuda, db, feats[:4], 3, 2, precision="fp8")
    assert e.value.code == hloc.EUNSUPPORTED
    db.close()


# ------------------------------------------------------------- scheduling shapes
def test_many_regions_multi_kernel_schedule(torch_cuda):
    # more regions than the single-block scheduler holds in LDS (16384): the
    # count / scan / scatter / expand kernels build the schedule
    rng = np.random.default_rng(21)
    R, n, d = 20_000, 40_000, 16
    region_of = np.sort(rng.integers(0, R, size=n)).astype(np.int32)
    feats = rng.standard_normal((n, d)).astype(np.float32)
    xy = rng.uniform(0, 80, size=(n, 2))
    q = (feats[rng.integers(0, n, 300)] + 0.2 * rng.standard_normal((300, d))).astype(np.float32)
    st, info, _ = check_all(torch_cuda, feats, xy, region_of, R, q, 5, 8,
                            name="20000 regions (multi-kernel schedule)")
    assert st["recall"] == 1.0 and info["items"] > 0


@pytest.mark.parametrize("precision,d", [("fp32", 64), ("bf16", 64), ("fp8", 64),
                                         ("bf16", 512), ("fp8", 512)])
def test_region_kept_by_every_frame(torch_cuda, precision, d):
    # one large region kept by all 700 frames (one wide item holds up to 1,024
    # frames): 47 row chunks of work items expanded from a single region; at
    # d = 512 the low-precision screens take wide chunks of 128 rows with the
    # rows in registers (3000 = 23 x 128 + 56: a ragged last chunk), 700
    # frames = 43 groups of 16 + 12
    rng = np.random.default_rng(22)
    sizes = np.array([3000] + [250] * 12)
    region_of = np.repeat(np.arange(len(sizes)), sizes).astype(np.int32)
    n = len(region_of)
    feats = rng.standard_normal((n, d)).astype(np.float32)
    feats[:3000] *= 0.2  # the big region sits near the origin, close to every query,
    feats[3000:] += 0.6  # the others are shifted away from it
    xy = rng.uniform(0, 40, size=(n, 2))
    q = (feats[rng.integers(0, 3000, 700)] + 0.05 * rng.standard_normal((700, d))).astype(np.float32)
    st, info, _ = check_all(torch_cuda, feats, xy, region_of, len(sizes), q, 9, 3,
                            name=f"one region kept by 700 frames, d {d}", precision=precision)
    assert st["recall"] == 1.0
    assert info["items"] >= (24 if d == 512 and precision != "fp32" else 47)


@pytest.mark.parametrize("d", [256, 512])
def test_wide_items_long_rows(torch_cuda, d):
    # wide items at the lengths where the fp32 wide kernel loads the next
    # frame group's operand ahead (256) and where it does not (512)
    rng = np.random.default_rng(24)
    sizes = np.array([700] + [90] * 10)
    region_of = np.repeat(np.arange(len(sizes)), sizes).astype(np.int32)
    n = len(region_of)
    feats = rng.standard_normal((n, d)).astype(np.float32)
    feats[:700] *= 0.2
    feats[700:] += 0.3
    xy = rng.uniform(0, 40, size=(n, 2))
    q = (feats[rng.integers(0, 700, 90)] + 0.05 * rng.standard_normal((90, d))).astype(np.float32)
    st, info, _ = check_all(torch_cuda, feats, xy, region_of, len(sizes), q, 9, 2,
                            name=f"one region kept by 90 frames, d{d}")
    assert st["recall"] == 1.0
    assert info["items"] > info["narrow_items"]


@pytest.mark.parametrize("precision", ["fp8", "bf16"])
def test_band_in_chunks(torch_cuda, precision):
    # rows all about equally far from the frames: the low-precision screen's
    # certificate fails and its band holds more rows than one pass fits, so
    # the band is re-scored in chunks (still exact)
    rng = np.random.default_rng(25)
    n, d = 6000, 64
    base = rng.standard_normal(d)
    feats = (base + 0.02 * rng.standard_normal((n, d))).astype(np.float32)
    region_of = (np.arange(n) // 1500).astype(np.int32)
    xy = rng.uniform(0, 40, size=(n, 2))
    q = (base + 0.02 * rng.standard_normal((20, d))).astype(np.float32)
    st, info, _ = check_all(torch_cuda, feats, xy, region_of, 4, q, 16, 2,
                            name=f"band in chunks, {precision}", precision=precision)
    assert st["recall"] == 1.0
    assert info["chunked_bands"] > 0 and info["band_rows"] > 1024


def test_statistics_follow_the_last_batch(torch_cuda):
    # the fine select writes one statistics record per frame and the info
    # call sums those of the last batch: after a large batch with chunked
    # bands, a small batch reports exactly what it reports on a fresh
    # database, and the counts are consistent with each other
    rng = np.random.default_rng(25)
    n, d = 6000, 64
    base = rng.standard_normal(d)
    feats = (base + 0.02 * rng.standard_normal((n, d))).astype(np.float32)
    region_of = (np.arange(n) // 1500).astype(np.int32)
    xy = rng.uniform(0, 40, size=(n, 2))
    big = (base + 0.02 * rng.standard_normal((40, d))).astype(np.float32)
    small = feats[[17, 2222, 4100]] + 1e-3 * rng.standard_normal((3, d)).astype(np.float32)
    keys = ("fine_fallbacks", "max_blocks", "chunked_bands", "band_rows", "rerank_rows",
            "candidates")
    fresh = make_db(feats, xy, region_of, 4, mirrors=hloc.MIRROR_FP8)
    run_device(torch_cuda, fresh, small, 16, 2, precision="fp8")
    want = fresh.info()
    fresh.close()
    db = make_db(feats, xy, region_of, 4, mirrors=hloc.MIRROR_FP8)
    run_device(torch_cuda, db, big, 16, 2, precision="fp8")
    first = db.info()
    run_device(torch_cuda, db, small, 16, 2, precision="fp8")
    got = db.info()
    say(f"[ok] large batch {first}; small batch {got}")
    assert first["chunked_bands"] > 0
    for info, nq in ((first, len(big)), (got, len(small))):
        assert info["chunked_bands"] <= info["fine_fallbacks"] <= nq
        assert info["band_rows"] <= info["rerank_rows"]
        assert 0 < info["max_blocks"]
    assert {k: got[k] for k in keys} == {k: want[k] for k in keys}
    db.close()


# ------------------------------------------------------------- tiles and the tuner
def test_tiles_do_not_change_results(torch_cuda, tmp_path):
    # the fine-screen tiles change the work items, never the results
    torch = torch_cuda
    w = workload.make_workload(1, nq=128)
    db = make_db(w.feats, w.xy, w.region_of, w.n_regions_total, w.agg)
    say("[case] results under every tile choice, then the tuner")
    ref = run_device(torch, db, w.q, w.k, w.n_reg)
    for rows, blocks in ((16, 2), (32, 16), (48, 4), (64, 8), (96, 8), (128, 16)):
        db.set_tiles(rows, blocks)
        assert db.tiles() == dict(rows_per_item=rows, blocks_per_cu=blocks)
        out = run_device(torch, db, w.q, w.k, w.n_reg)
        for key in ref:
            assert out[key].tobytes() == ref[key].tobytes(), (rows, blocks, key)
    for bad in ((144, 8), (24, 8), (0, 8), (64, 0), (64, 33)):
        with pytest.raises(hloc.HlocError) as e:
            db.set_tiles(*bad)
        assert e.value.code == hloc.EINVAL
    qd = torch.from_numpy(w.q).to("cuda:0")
    cache = str(tmp_path / "tiles.json")
    t1 = db.autotune(qd, w.k, w.n_reg, cache=cache, reps=2)
    assert t1["source"] == "tuned" and t1["rows_per_item"] in (32, 64, 96, 128)
    assert db.tiles() == dict(rows_per_item=t1["rows_per_item"], blocks_per_cu=t1["blocks_per_cu"])
    t2 = db.autotune(qd, w.k, w.n_reg, cache=cache)
    assert t2["source"] == "cache" and t2["rows_per_item"] == t1["rows_per_item"]
    out = run_device(torch, db, w.q, w.k, w.n_reg)
    for key in ref:
        assert out[key].tobytes() == ref[key].tobytes(), key
    say(f"[ok] tuner chose {t1}")
    db.close()


@pytest.mark.parametrize("rows", [16, 32, 128])
def test_wide_items_with_short_chunks(torch_cuda, rows):
    # the wide kernel stages chunks of fewer than 64 rows too; with 128-row
    # tiles the narrow items take 128 rows and the wide ones 64
    rng = np.random.default_rng(23)
    sizes = np.array([1000] + [120] * 8)
    region_of = np.repeat(np.arange(len(sizes)), sizes).astype(np.int32)
    n, d = len(region_of), 64
    feats = rng.standard_normal((n, d)).astype(np.float32)
    feats[:1000] *= 0.2
    feats[1000:] += 0.6
    xy = rng.uniform(0, 40, size=(n, 2))
    q = (feats[rng.integers(0, 1000, 300)] + 0.05 * rng.standard_normal((300, d))).astype(np.float32)
    say(f"[case] 300 frames on one region, {rows}-row chunks")
    db = make_db(feats, xy, region_of, len(sizes), mirrors=hloc.MIRROR_BF16)
    db.set_tiles(rows, 8)
    for precision in ("fp32", "bf16"):
        out = run_device(torch_cuda, db, q, 9, 2, precision=precision)
        regs = db.last_regions()
        info = db.info()
        ora = oracle.localize(feats, xy, region_of, len(sizes), q, np.arange(len(q) + 1), 9, 2,
                              (0.5, 1, 0.0, 0))
        st = judge_frames(out["idx"], out["dist"], regs, ora, feats, region_of, len(sizes), q, 9)
        say(f"[ok] {precision}: {st} info={info}")
        assert st["recall"] == 1.0 and info["items"] > info["narrow_items"]
    db.close()

