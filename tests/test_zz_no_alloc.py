"""The entry point that allocates nothing (hloc_query_batch_static_async),
through the C ABI: two calls in a row on one device, the second smaller, so
it runs on the static array as the first call left it. Each must give the
results of hloc_query_batch_async bit for bit (and those are judged against
the FP64 oracle by the parity tests; the smaller call is judged here too).
A batch whose scratch would exceed the array is refused on the host."""
import os
import sys

import numpy as np
import pytest

import oracle
from parity import judge_frames, judge_requests
from paper_2006_08861_amd import hloc, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(hloc.LIB_PATH):
        pytest.fail("libhloc.so is not built")
    w = workload.make_workload(1)
    db = hloc.HlocDB(w.feats, w.xy, mirrors=hloc.MIRROR_BF16 | hloc.MIRROR_FP8)
    db.set_regions(w.region_of, w.n_regions_total)
    db.set_aggregation(*w.agg)
    yield torch, w, db
    db.close()


def both(torch, db, q, k, n_reg, offs, precision):
    qd = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to("cuda:0")
    od = None if offs is None else torch.from_numpy(np.asarray(offs, np.int32)).to("cuda:0")
    a = db.query_static(qd, k, n_reg, od, precision=precision)
    torch.cuda.synchronize()
    a = {key: v.cpu().numpy() for key, v in a.items()}
    b = db.query(qd, k, n_reg, od, precision=precision)
    torch.cuda.synchronize()
    b = {key: v.cpu().numpy() for key, v in b.items()}
    for key in ("idx", "dist", "xy", "tile", "flags"):
        assert a[key].tobytes() == b[key].tobytes(), f"{key} differs from hloc_query_batch_async"
    return a


def test_static_entry_two_calls_second_smaller(setup):
    torch, w, db = setup
    say(f"[case] static entry, call 1: {len(w.q)} frames, k {w.k}, n_regions {w.n_reg}, fp32")
    both(torch, db, w.q, w.k, w.n_reg, w.req_offsets, "fp32")
    # call 2: 37 frames in ragged requests of 1..5 frames, k 8, bf16 screen
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(len(w.q), 37, replace=False))
    q = w.q[sel]
    sizes = [1, 5, 2, 3, 4, 1, 5, 3, 2, 4, 3, 4]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    assert offs[-1] == len(q)
    say(f"[case] static entry, call 2: {len(q)} frames in {len(sizes)} requests, k 8, bf16")
    res = both(torch, db, q, 8, w.n_reg, offs, "bf16")
    reps, _ = oracle.region_means(w.feats, w.region_of, w.n_regions_total)
    ora = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, q, 8, w.n_reg, reps=reps)
    st = judge_frames(res["idx"], res["dist"], None, ora, w.feats, w.region_of,
                      w.n_regions_total, q, 8, reps=reps)
    tile, pos, flags = [], [], []
    for r in range(len(sizes)):
        ix, iy, x, y, fl = oracle.aggregate(ora["idx"][offs[r]:offs[r + 1]].ravel(), w.xy, *w.agg)
        tile.append((ix, iy))
        pos.append((x, y))
        flags.append(fl)
    ora.update(tile=np.asarray(tile), pos=np.asarray(pos), flags=np.asarray(flags))
    same = judge_requests(res["idx"], res["xy"], res["tile"], res["flags"], ora, w.xy, offs, w.agg)
    say(f"[ok] {st} same_pools={same}/{len(sizes)}")
    assert st["recall"] == 1.0


def test_static_entry_refuses_large_batch(setup):
    torch, w, db = setup
    # 20,000 frames against 1,024 regions: the coarse words alone take 82 MB
    q = torch.zeros((20000, w.feats.shape[1]), dtype=torch.float32, device="cuda:0")
    with pytest.raises(hloc.HlocError) as e:
        db.query_static(q, w.k, w.n_reg)
    assert e.value.code == hloc.EINVAL and "static" in str(e.value)
    torch.cuda.synchronize()
