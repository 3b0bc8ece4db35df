"""The request server (hloc_server_*): continuous batching of 1-16 frame
requests on several batches in flight. Each request's results must be the
same alone (one hloc_query_batch call) and in the mix, and match the FP64
oracle under the acceptance rule."""
import threading
import time

import numpy as np
import pytest

import oracle
from parity import judge_frames
from paper_2006_08861_amd import hloc, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def serve_db():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = workload.make_workload(4, nq=48, n=30_000)
    db = hloc.HlocDB(w.feats, w.xy)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    yield w, db
    db.close()


def _requests(w, rng, count):
    """(frames, k) of `count` requests of 1-16 frames taken from the workload's
    requests, each with k in {8, 16, 32}."""
    out = []
    offs = w.req_offsets
    for i in range(count):
        r = i % (len(offs) - 1)
        out.append((w.q[offs[r]:offs[r + 1]], int(rng.choice([8, 16, 32]))))
    return out


def test_server_results_same_alone_and_in_the_mix(serve_db):
    w, db = serve_db
    rng = np.random.default_rng(31)
    reqs = _requests(w, rng, 72)
    say(f"[case] server: {len(reqs)} requests of 1-16 frames, 4 submitting threads, 3 slots")
    srv = hloc.Server(db, k=32, n_regions=w.n_reg, max_batch_frames=64, max_slots=3,
                      max_queue_frames=4096)
    results = [None] * len(reqs)
    errors = []

    def client(ids):
        try:
            local = np.random.default_rng(ids[0])
            pending = []
            for i in ids:
                frames, k = reqs[i]
                pending.append((i, srv.submit(frames, k)))
                time.sleep(float(local.uniform(0, 0.002)))
            for i, t in pending:
                results[i] = srv.wait(t, len(reqs[i][0]), reqs[i][1])
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=client, args=(list(range(j, len(reqs), 4)),))
               for j in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    st = srv.stats()
    srv.close()
    say(f"[ok] server stats {st}")
    assert st["requests"] == len(reqs) and st["frames"] == sum(len(f) for f, _ in reqs)
    for i, (frames, k) in enumerate(reqs):
        alone = db.query(frames, k, w.n_reg, np.array([0, len(frames)], np.int32))
        got = results[i]
        np.testing.assert_array_equal(got["idx"], alone["idx"])
        np.testing.assert_array_equal(got["dist"].view(np.uint32), alone["dist"].view(np.uint32))
        np.testing.assert_array_equal(got["xy"].view(np.uint64), alone["xy"][0].view(np.uint64))
        np.testing.assert_array_equal(got["tile"], alone["tile"][0])
        assert got["flags"] == int(alone["flags"][0])
        assert got["latency_ms"] > 0
    # and the mixed results against the oracle, frame by frame
    for k in (8, 16, 32):
        sel = [i for i, (_, kk) in enumerate(reqs) if kk == k][:6]
        q = np.concatenate([reqs[i][0] for i in sel])
        idx = np.concatenate([results[i]["idx"] for i in sel])
        dist = np.concatenate([results[i]["dist"] for i in sel])
        ora = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, q,
                              np.arange(len(q) + 1), k, w.n_reg, w.agg)
        st_k = judge_frames(idx, dist, np.asarray(ora["regions"]), ora, w.feats, w.region_of,
                            w.n_regions_total, q, k)
        say(f"[ok] k={k}: {st_k}")
        assert st_k["recall"] == 1.0


def test_server_admission_and_limits(serve_db):
    w, db = serve_db
    say("[case] server admission by HBM budget and queue limits")
    with pytest.raises(hloc.HlocError) as e:
        hloc.Server(db, k=16, n_regions=w.n_reg, max_batch_frames=64, hbm_budget_bytes=1024)
    assert e.value.code == hloc.ENOMEM
    probe = hloc.Server(db, k=16, n_regions=w.n_reg, max_batch_frames=64, max_slots=1)
    slot = probe.stats()["slot_bytes"]
    probe.close()
    srv = hloc.Server(db, k=16, n_regions=w.n_reg, max_batch_frames=16, max_slots=8,
                      max_queue_frames=16, hbm_budget_bytes=2 * slot)
    st = srv.stats()
    assert st["slots"] >= 2  # a 16-frame slot is smaller than a 64-frame one
    frames = w.q[:16]
    with pytest.raises(hloc.HlocError) as e:
        srv.submit(w.q[:17])
    assert e.value.code == hloc.EINVAL
    with pytest.raises(hloc.HlocError) as e:
        srv.submit(frames, k=17)
    assert e.value.code == hloc.EINVAL
    tickets, refused = [], 0
    for _ in range(40):
        try:
            tickets.append(srv.submit(frames, 16))
        except hloc.HlocError as err:
            assert err.code == hloc.EBUSY
            refused += 1
    outs = [srv.wait(t, 16, 16) for t in tickets]
    st = srv.stats()
    assert st["refused"] == refused and st["requests"] == len(tickets)
    assert st["peak_queued_frames"] <= 16
    for o in outs[1:]:
        np.testing.assert_array_equal(o["idx"], outs[0]["idx"])
    with pytest.raises(hloc.HlocError) as e:
        srv.wait(tickets[0], 16, 16)  # released by the first wait
    assert e.value.code == hloc.EINVAL
    with pytest.raises(hloc.HlocError) as e:
        db.set_aggregation(*w.agg)  # read-only while a server exists
    assert e.value.code == hloc.ESTATE
    srv.close()
    db.set_aggregation(*w.agg)
    say(f"[ok] slots={st['slots']} refused={refused} served={len(tickets)}")
