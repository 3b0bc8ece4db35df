"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
exact rational brute force on tiny inputs, a library k-d tree for the
exhaustive case, exact-match queries, permutation invariance, closed forms of
the representatives, and hand-worked aggregation cases (tests/golden)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- brute force
def _brute(feats, region_of, R, q, k, n_reg):
    """Exact rational two-stage search: region means and squared distances as
    Fractions, ranks by (d2, id) with Python's sorted()."""
    n, d = len(feats), len(feats[0])
    F = [[Fraction(v) for v in row] for row in feats]
    Q = [Fraction(v) for v in q]
    members = {r: [j for j in range(n) if region_of[j] == r] for r in range(R)}
    reps = {}
    for r, js in members.items():
        if js:
            reps[r] = [sum(F[j][i] for j in js) / len(js) for i in range(d)]
    rd = sorted((sum((Q[i] - c[i]) ** 2 for i in range(d)), r) for r, c in reps.items())
    kept = [r for _, r in rd[:n_reg]]
    cand = sorted((sum((Q[i] - F[j][i]) ** 2 for i in range(d)), j)
                  for r in kept for j in members[r])
    top = cand[:k]
    idx = [j for _, j in top] + [-1] * (k - len(top))
    dist = [float(v) for v, _ in top] + [math.inf] * (k - len(top))
    return sorted(kept), idx, dist


def _dyadic_case(rng, n, d, R):
    # quarter-integers in [-2, 2] and power-of-two region sizes: every mean,
    # difference, square and sum is exact in FP64, so the oracle must agree
    # with exact arithmetic bit for bit, tie order included
    feats = rng.integers(-8, 9, size=(n, d)) / 4.0
    sizes = []
    left = n
    while left:
        s = int(rng.choice([v for v in (1, 2, 4) if v <= left]))
        sizes.append(s)
        left -= s
    region_of = np.repeat(np.arange(len(sizes)), sizes)
    perm = rng.permutation(n)  # regions need not be contiguous
    return feats[perm], region_of, len(sizes)


@pytest.mark.parametrize("seed", range(40))
def test_two_stage_matches_exact_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n, d = int(rng.integers(1, 13)), int(rng.integers(1, 5))
    feats, region_of, R = _dyadic_case(rng, n, d, 0)
    q = rng.integers(-8, 9, size=d) / 4.0
    k = int(rng.integers(1, 7))
    n_reg = int(rng.integers(1, R + 2))
    kept, idx, dist = _brute(feats.tolist(), region_of.tolist(), R, q.tolist(), k, n_reg)
    res = oracle.retrieve(feats, region_of, R, q[None, :], k, n_reg)
    assert sorted(res["regions"][0].tolist()) == kept
    assert res["idx"][0].tolist() == idx
    assert res["d2"][0].tolist() == dist


@pytest.mark.parametrize("seed", range(10))
def test_float_inputs_match_bruteforce(seed):
    # generic float32 data: distances agree with exact arithmetic to FP64
    # rounding, and (ties being improbable) the index lists are identical
    rng = np.random.default_rng(100 + seed)
    n, d, R = 12, 4, 4
    feats = rng.standard_normal((n, d)).astype(np.float32)
    region_of = rng.integers(0, R, size=n)
    q = rng.standard_normal(d).astype(np.float32)
    kept, idx, dist = _brute(feats.astype(np.float64).tolist(), region_of.tolist(), R,
                             q.astype(np.float64).tolist(), 5, 2)
    res = oracle.retrieve(feats, region_of, R, q[None, :], 5, 2)
    assert sorted(res["regions"][0].tolist()) == kept
    assert res["idx"][0].tolist() == idx
    np.testing.assert_allclose(res["d2"][0][np.isfinite(dist)], np.array(dist)[np.isfinite(dist)],
                               rtol=1e-14)


def test_exhaustive_equals_kdtree():
    # n_reg = R is the paper's whole-database search: a textbook kNN
    rng = np.random.default_rng(7)
    n, d, R, k = 3000, 16, 37, 12
    feats = rng.standard_normal((n, d)).astype(np.float32)
    region_of = rng.integers(0, R, size=n)
    qs = rng.standard_normal((25, d)).astype(np.float32)
    res = oracle.retrieve(feats, region_of, R, qs, k, R)
    dd, ii = cKDTree(feats.astype(np.float64)).query(qs.astype(np.float64), k=k)
    for i in range(len(qs)):
        assert set(res["idx"][i].tolist()) == set(ii[i].tolist())
        np.testing.assert_allclose(np.sqrt(res["d2"][i]), dd[i], rtol=1e-12)


def test_one_region_per_row_reduces_to_knn():
    # every row its own region: the coarse level already ranks rows, so
    # keeping k regions returns the exhaustive top k
    rng = np.random.default_rng(8)
    n, d, k = 400, 8, 6
    feats = rng.standard_normal((n, d))
    qs = rng.standard_normal((10, d))
    res = oracle.retrieve(feats, np.arange(n), n, qs, k, k)
    _, ii = cKDTree(feats).query(qs, k=k)
    for i in range(len(qs)):
        assert res["idx"][i].tolist() == ii[i].tolist()
        assert sorted(res["regions"][i].tolist()) == sorted(ii[i].tolist())


def test_exact_match_query_gives_zero_and_self():
    rng = np.random.default_rng(9)
    n, d, R = 500, 32, 10
    feats = rng.standard_normal((n, d)).astype(np.float32)
    region_of = rng.integers(0, R, size=n)
    js = rng.integers(0, n, size=20)
    res = oracle.retrieve(feats, region_of, R, feats[js], 3, R)
    assert (res["idx"][:, 0] == js).all()
    assert (res["d2"][:, 0] == 0.0).all()
    assert (res["d2"][:, 1] > 0.0).all()
    # with pruning the self match survives whenever its region is kept
    res = oracle.retrieve(feats, region_of, R, feats[js], 3, 2)
    for i, j in enumerate(js):
        if region_of[j] in res["regions"][i]:
            assert res["idx"][i, 0] == j and res["d2"][i, 0] == 0.0


def test_database_permutation_invariance():
    rng = np.random.default_rng(10)
    n, d, R, k = 800, 12, 16, 9
    feats = rng.standard_normal((n, d)).astype(np.float32)
    region_of = rng.integers(0, R, size=n)
    qs = rng.standard_normal((15, d)).astype(np.float32)
    perm = rng.permutation(n)
    a = oracle.retrieve(feats, region_of, R, qs, k, 4)
    b = oracle.retrieve(feats[perm], region_of[perm], R, qs, k, 4)
    np.testing.assert_array_equal(a["d2"], b["d2"])
    np.testing.assert_array_equal(a["idx"], perm[b["idx"]])


def test_representatives_closed_forms():
    rng = np.random.default_rng(11)
    feats = rng.standard_normal((6, 5)).astype(np.float32)
    feats[3] = feats[4] = feats[5]
    region_of = np.array([0, 1, 1, 2, 2, 2])
    reps, nz = oracle.region_means(feats, region_of, 4)
    np.testing.assert_array_equal(reps[0], feats[0].astype(np.float64))   # one member
    np.testing.assert_array_equal(reps[2], feats[5].astype(np.float64))   # identical members
    np.testing.assert_allclose(reps[1], (feats[1].astype(np.float64) + feats[2]) / 2, rtol=0)
    assert nz.tolist() == [True, True, True, False]
    assert np.isnan(reps[3]).all()


def test_empty_region_never_selected():
    feats = np.array([[0.0], [1.0], [5.0]])
    res = oracle.retrieve(feats, np.array([0, 0, 2]), 3, np.array([[0.4]]), 2, 3)
    assert sorted(res["regions"][0].tolist()) == [0, 2]


def test_padding_when_fewer_candidates_than_k():
    feats = np.array([[0.0, 0.0], [3.0, 4.0], [10.0, 0.0]])
    res = oracle.retrieve(feats, np.array([0, 0, 1]), 2, np.array([[0.0, 0.0]]), 4, 1)
    assert res["idx"][0].tolist() == [0, 1, -1, -1]
    assert res["d2"][0].tolist() == [0.0, 25.0, math.inf, math.inf]
    assert res["n_cand"][0] == 2


def test_gap_and_tie_band():
    # rows at squared distances 1, 4, 4, 9 from q: the k=2 boundary is an
    # exact tie (gap 0) and both tied rows are in the band; k=3 has gap 5/9
    feats = np.array([[1.0, 0.0], [0.0, 2.0], [2.0, 0.0], [0.0, -3.0]])
    q = np.array([[0.0, 0.0]])
    r2 = oracle.retrieve(feats, np.zeros(4, int), 1, q, 2, 1)
    assert r2["idx"][0].tolist() == [0, 1] and r2["gap_k"][0] == 0.0
    assert sorted(r2["band"][0][0].tolist()) == [1, 2]
    r3 = oracle.retrieve(feats, np.zeros(4, int), 1, q, 3, 1)
    assert r3["gap_k"][0] == pytest.approx(5.0 / 9.0, rel=1e-15)


def test_tile_floor_exact_on_dyadic_cell():
    rng = np.random.default_rng(12)
    xy = rng.uniform(-50, 50, size=(2000, 2))
    t = oracle.tile_of(xy, 0.5)
    for (x, y), (ix, iy) in zip(xy.tolist(), t.tolist()):
        assert ix == math.floor(Fraction(x) / Fraction(1, 2))
        assert iy == math.floor(Fraction(y) / Fraction(1, 2))


# ---------------------------------------------------------------- aggregation
def _load_cases():
    with open(os.path.join(GOLDEN, "aggregation_cases.json")) as f:
        return json.load(f)["cases"]


def _case_inputs(case):
    cell = case["cell"]
    if "tiles" in case:
        pts, rows = [], []
        for ix, iy, c in case["tiles"]:
            rows += [len(pts)] * c
            pts.append([(ix + 0.5) * cell, (iy + 0.5) * cell])
        return np.array(pts), np.array(rows)
    pts = np.array(case["points"], dtype=np.float64)
    rows = np.array(case.get("rows", list(range(len(pts)))))
    return pts, rows


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: c["name"])
def test_aggregation_golden(case):
    xy, rows = _case_inputs(case)
    ix, iy, x, y, flag = oracle.aggregate(rows, xy, case["cell"], case["top_c"], case["radius"],
                                          case["toler_pct"])
    assert [ix, iy] == case["expect"]["tile"]
    assert flag == case["expect"]["flag"]
    if flag == oracle.FLAG_EMPTY:
        assert math.isnan(x) and math.isnan(y)
    if "pos" in case["expect"]:
        assert [x, y] == case["expect"]["pos"]


def test_aggregation_shuffle_invariant():
    # the estimate depends on the multiset of candidates, not their order
    rng = np.random.default_rng(13)
    for case in _load_cases():
        xy, rows = _case_inputs(case)
        a = oracle.aggregate(rows, xy, case["cell"], case["top_c"], case["radius"], case["toler_pct"])
        b = oracle.aggregate(rng.permutation(rows), xy, case["cell"], case["top_c"], case["radius"],
                             case["toler_pct"])
        assert a[:2] == b[:2] and a[4] == b[4]


def test_multiframe_pooling_counts_every_frame():
    # two requests; the second repeats one frame three times, so its pooled
    # candidates are three copies of that frame's list
    rng = np.random.default_rng(14)
    feats = rng.standard_normal((300, 6))
    xy = rng.uniform(0, 30, size=(300, 2))
    q = rng.standard_normal((4, 6))
    q[2] = q[3] = q[1]
    res = oracle.localize(feats, xy, np.zeros(300, int), 1, q, [0, 1, 4], 5, 1, (0.5, 1, 0.0, 0))
    pooled = res["idx"][1:4].ravel()
    assert sorted(pooled.tolist()) == sorted(res["idx"][1].tolist() * 3)
    ix, iy, _, _, _ = oracle.aggregate(pooled, xy, 0.5, 1, 0.0, 0)
    assert res["tile"][1].tolist() == [ix, iy]


def test_localize_recovers_synthetic_position():
    # the whole path on a small synthetic corridor database puts most
    # estimates near where the queries were drawn (a sanity check of the
    # workload, not a pin of the arithmetic)
    from paper_2006_08861_amd import workload
    w = workload.make_workload(0, nq=100)
    res = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q, w.req_offsets,
                          w.k, w.n_reg, w.agg)
    err = np.linalg.norm(res["pos"] - w.xy[w.truth], axis=1)
    assert np.median(err) < 1.0 and np.mean(err < 2.5) > 0.9


def test_duplicates_across_frames_change_the_estimate():
    # frame A returns rows 0-2 (tile (0,0)); frame B, sent twice, returns rows
    # 3-5 (tile (5,5)). Counting every return gives (5,5) 6 votes to 3; a
    # de-duplicated pool would tie 3:3 and pick (0,0) by the (iy, ix) order.
    feats = np.array([[0, 0], [0, 0.1], [0, 0.2], [10, 0], [10, 0.1], [10, 0.2], [50, 50]],
                     dtype=np.float64)
    xy = np.array([[0.25, 0.25]] * 3 + [[2.75, 2.75]] * 3 + [[40.0, 40.0]])
    q = np.array([[0, 0.05], [10, 0.05], [10, 0.05]])
    res = oracle.localize(feats, xy, np.zeros(7, int), 1, q, [0, 3], 3, 1, (0.5, 1, 0.0, 0))
    assert res["tile"][0].tolist() == [5, 5]
    assert res["pos"][0].tolist() == [2.75, 2.75]


def test_window_requests_hand_case():
    # the duplicates case above as windows over two distinct frames: request
    # 0 = frames (A, B, B) votes (5,5) 6:3; request 1 = frames (A) alone
    # votes (0,0); request 2 = (B, A) ties 3:3 and takes (0,0) by (iy, ix)
    feats = np.array([[0, 0], [0, 0.1], [0, 0.2], [10, 0], [10, 0.1], [10, 0.2], [50, 50]],
                     dtype=np.float64)
    xy = np.array([[0.25, 0.25]] * 3 + [[2.75, 2.75]] * 3 + [[40.0, 40.0]])
    q = np.array([[0, 0.05], [10, 0.05]])
    res = oracle.localize(feats, xy, np.zeros(7, int), 1, q, [0, 3, 4, 6], 3, 1,
                          (0.5, 1, 0.0, 0), req_frames=[0, 1, 1, 0, 1, 0])
    assert res["tile"].tolist() == [[5, 5], [0, 0], [0, 0]]


def test_sliding_windows_equal_materialised_requests():
    # windows of M = 5 consecutive frames over a walk of 40 frames (each
    # frame retrieved once) give the same estimates as sending every
    # window's frames again as its own request
    from paper_2006_08861_amd import workload
    w = workload.make_workload(0, nq=40)
    M = 5
    starts = np.arange(0, len(w.q) - M + 1)
    frames = np.concatenate([np.arange(s0, s0 + M) for s0 in starts])
    offs = np.arange(len(starts) + 1) * M
    agg = (0.3, 10, 3.0, 20)
    win = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q, offs, w.k,
                          w.n_reg, agg, req_frames=frames)
    mat = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q[frames], offs, w.k,
                          w.n_reg, agg)
    assert win["tile"].tolist() == mat["tile"].tolist()
    assert win["flags"].tolist() == mat["flags"].tolist()
    ident = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q, [0, 7, 40], w.k,
                            w.n_reg, agg, req_frames=np.arange(40))
    plain = oracle.localize(w.feats, w.xy, w.region_of, w.n_regions_total, w.q, [0, 7, 40], w.k,
                            w.n_reg, agg)
    assert ident["tile"].tolist() == plain["tile"].tolist()


def test_labels_single_label_is_localize():
    w = workload_small()
    R = w.n_regions_total
    one = oracle.localize_labels(w.feats, w.xy, w.region_of, R, np.zeros(R, int), w.q,
                                 w.req_offsets, w.k, w.n_reg, w.agg)
    plain = oracle.localize(w.feats, w.xy, w.region_of, R, w.q, w.req_offsets, w.k, w.n_reg,
                            w.agg)
    assert np.array_equal(one["idx"][0], plain["idx"])
    assert one["tile"].tolist() == plain["tile"].tolist()


def test_labels_equal_sub_databases():
    # label p's lists are the plain search over a database holding only the
    # rows of label p's regions (row ids mapped back), and hold only such rows
    w = workload_small()
    R = w.n_regions_total
    labels = (np.arange(R) * 3) // R  # three contiguous runs of regions (paths)
    res = oracle.localize_labels(w.feats, w.xy, w.region_of, R, labels, w.q, w.req_offsets,
                                 w.k, w.n_reg, w.agg)
    for p in range(3):
        rows = np.nonzero(labels[w.region_of] == p)[0]
        sub = oracle.retrieve(w.feats[rows], w.region_of[rows], R, w.q, w.k, w.n_reg)
        mapped = np.where(sub["idx"] >= 0, rows[np.maximum(sub["idx"], 0)], -1)
        assert np.array_equal(mapped, res["idx"][p]), p
        got = res["idx"][p][res["idx"][p] >= 0]
        assert np.all(labels[w.region_of[got]] == p)
    # a request pools frames x labels x k candidates
    i = 0
    f0, f1 = w.req_offsets[i], w.req_offsets[i + 1]
    pooled = res["idx"][:, f0:f1].transpose(1, 0, 2).ravel()
    ix, iy, _, _, _ = oracle.aggregate(pooled, w.xy, *w.agg)
    assert res["tile"][i].tolist() == [ix, iy]
    assert len(pooled) == (f1 - f0) * 3 * w.k


def workload_small():
    from paper_2006_08861_amd import workload
    return workload.make_workload(0, nq=24)


# ------------------------------------------------ FFT-magnitude feature pins
def test_fft_magnitude_hand_case():
    # x = (1, 2, 3, 4): X_0 = 10, X_1 = -2 + 2i, X_2 = -2 (worked by hand)
    got = oracle.fft_magnitude([[1.0, 2.0, 3.0, 4.0]], 3)
    assert np.allclose(got, [[10.0, 2.0 * math.sqrt(2.0), 2.0]], rtol=1e-15, atol=1e-14)
    # L = 2: X_0 = x0 + x1, X_1 = x0 - x1
    assert np.allclose(oracle.fft_magnitude([[3.0, -5.0]], 2), [[2.0, 8.0]], rtol=0, atol=1e-14)


def test_fft_magnitude_matches_library_transform():
    """The definition written out agrees with numpy's fast real transform."""
    rng = np.random.default_rng(7)
    for L in (2, 3, 8, 12, 64, 512):
        x = rng.standard_normal((5, L)) * 10
        d = L // 2 + 1
        lib = np.abs(np.fft.rfft(x, axis=1))[:, :d]
        got = oracle.fft_magnitude(x, d)
        assert np.allclose(got, lib, rtol=0, atol=1e-11 * np.abs(x).sum()), L


def test_fft_magnitude_tones_and_constant():
    """A constant c gives |c| L in bin 0 only; A cos(2 pi m t / L + phi) gives
    A L / 2 in bin m only (0 < m < L/2)."""
    L, d = 256, 129
    t = np.arange(L)
    const = oracle.fft_magnitude(np.full((1, L), -2.5), d)[0]
    assert abs(const[0] - 2.5 * L) < 1e-10 and np.all(const[1:] < 1e-10)
    for m, A, phi in ((1, 3.0, 0.3), (17, 0.5, -1.1), (127, 7.0, 2.0)):
        tone = oracle.fft_magnitude((A * np.cos(2 * np.pi * m * t / L + phi))[None], d)[0]
        assert abs(tone[m] - A * L / 2) < 1e-9, m
        rest = np.delete(tone, m)
        assert np.all(rest < 1e-9), m


def test_fft_magnitude_invariances():
    """Rotation of the panorama (circular shift), mirror (time reversal) and
    Parseval's identity over the half spectrum."""
    rng = np.random.default_rng(11)
    for L in (8, 96, 512):
        x = rng.standard_normal((4, L))
        d = L // 2 + 1
        f = oracle.fft_magnitude(x, d)
        for s in (1, L // 3, L - 1):
            assert np.allclose(oracle.fft_magnitude(np.roll(x, s, axis=1), d), f,
                               rtol=1e-12, atol=1e-12)
        mirrored = np.concatenate([x[:, :1], x[:, :0:-1]], axis=1)  # x_{-t mod L}
        assert np.allclose(oracle.fft_magnitude(mirrored, d), f, rtol=1e-12, atol=1e-12)
        w = np.full(d, 2.0)
        w[0] = 1.0
        if L % 2 == 0:
            w[-1] = 1.0
        assert np.allclose((f * f * w).sum(axis=1) / L, (x * x).sum(axis=1), rtol=1e-12)


def test_fft_magnitude_rejects_bad_shapes():
    with pytest.raises(ValueError):
        oracle.fft_magnitude([[1.0]], 1)
    with pytest.raises(ValueError):
        oracle.fft_magnitude([[1.0, 2.0, 3.0, 4.0]], 4)
    with pytest.raises(ValueError):
        oracle.fft_magnitude([[1.0, 2.0, 3.0, 4.0]], 0)
