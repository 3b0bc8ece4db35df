"""Plain CPU FP64 oracle for hierarchical L2 retrieval and 2-D aggregation.

TEST INFRASTRUCTURE. Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module. The product path never calls it; it
shares no code, table or constant generator with the HIP library.

What it computes, and where the method is stated
-------------------------------------------------
Hu, Zhu, Zhang, "GPU-accelerated Hierarchical Panoramic Image Feature Retrieval
for Indoor Localization" (ICMR 2016).

* Retrieval (Section 3.1, Algorithm 1; Section 4): every query frame is
  compared with database frames by Euclidean distance and the N candidates of
  smallest distance are kept per frame. The paper searches the whole database
  (all subspaces). The two-stage form computed here first ranks regions (runs of
  database rows) by the distance from the query to each region's mean vector
  and keeps the best `n_reg`, then searches every row of those regions. With
  `n_reg` equal to the number of non-empty regions it is exactly the paper's
  exhaustive search.
* Multi-frame retrieval (Section 3, Section 3.1): a request carries several
  frames; every frame is retrieved on its own and the candidates of all frames
  of the request are pooled, duplicates included (Section 4 notes that several
  frames may return the same location).
* Aggregation (Section 3.2, Algorithm 2): candidates are mapped to floor-plan
  coordinates, binned into square tiles, tiles are ranked by candidate count,
  and the first of the TopC best tiles whose tolerance circle holds more than
  tolerPer of all candidates is the location estimate.

* Omnidirectional feature (Section 3): the magnitude of the discrete Fourier
  transform of a 1-D panoramic signal, bins 0 .. d-1 (`fft_magnitude`).

Readings where the paper is silent (each repeated in the design notes):
distances are squared L2 (same ranking as Euclidean); ties rank by (d^2,
original row index) and regions by (d^2, region id); fewer than k candidates pad
with index -1 and distance +inf; an empty region is never selected; tiles are
floor(coord / cell) from origin (0, 0); tiles rank by (count desc, iy asc, ix
asc); the tolerance circle holds the tiles whose integer tile offset (dx, dy)
has dx^2 + dy^2 <= rho^2 with rho = round(radius / cell); the threshold test is
strict, 100 * circle > toler_pct * total, with total counting duplicates and
excluding padding; if no top tile passes the rank-1 tile is returned flagged
LOW_CONFIDENCE; the position returned is the tile centre ((ix + 0.5) * cell,
(iy + 0.5) * cell).

Everything is float64 with direct differences sum_i (q_i - f_i)^2; float32
inputs promote exactly.
"""
from __future__ import annotations

import math

import numpy as np

FLAG_LOW_CONFIDENCE = 1
FLAG_EMPTY = 2
TIE_REL = 1e-6


def _rel_gap(lo: float, hi: float) -> float:
    """Relative gap between two consecutive sorted distances (inf if absent)."""
    if not np.isfinite(hi):
        return math.inf
    return (hi - lo) / max(hi, 1e-300)


def region_means(feats: np.ndarray, region_of: np.ndarray, n_regions_total: int):
    """Mean vector of each region's rows in FP64 (the coarse representative).

    Returns (reps, nonempty): reps[r] is (1/s_r) * sum of the rows with
    region_of == r; rows of empty regions are NaN and nonempty[r] is False.
    """
    f = np.asarray(feats)  # float32 values are added to the FP64 sums exactly promoted
    reg = np.asarray(region_of, dtype=np.int64)
    d = f.shape[1]
    sums = np.zeros((n_regions_total, d), dtype=np.float64)
    np.add.at(sums, reg, f)
    counts = np.bincount(reg, minlength=n_regions_total).astype(np.int64)
    reps = np.full((n_regions_total, d), np.nan)
    nz = counts > 0
    reps[nz] = sums[nz] / counts[nz, None]
    return reps, nz


def sq_dist(q: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance from one vector q to each row, FP64 direct
    differences."""
    diff = np.asarray(rows, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return (diff * diff).sum(axis=1)


def select_regions(q: np.ndarray, reps: np.ndarray, nonempty: np.ndarray, n_reg: int):
    """Coarse level for one query: rank the non-empty regions by (d^2 to the
    representative, region id) and keep the first n_reg.

    Returns (region ids, their d^2, relative gap between the n_reg-th and the
    next region, inf if none follows).
    """
    ids = np.nonzero(nonempty)[0]
    d2 = sq_dist(q, reps[ids])
    order = np.lexsort((ids, d2))
    ids, d2 = ids[order], d2[order]
    m = min(n_reg, len(ids))
    gap = _rel_gap(d2[m - 1], d2[m]) if m < len(ids) else math.inf
    return ids[:m], d2[:m], gap


def search_rows(q: np.ndarray, feats: np.ndarray, rows: np.ndarray, k: int, tie_rel: float = TIE_REL):
    """Fine level for one query: squared L2 to each candidate row, ranked by
    (d^2, row index), first k kept (padded with -1 / +inf).

    Returns (idx[k], d2[k], gap at the k / k+1 boundary, tie band) where the
    tie band lists (row, d^2) of every candidate whose d^2 lies within
    tie_rel * d2_k of the k-th distance d2_k.
    """
    rows = np.asarray(rows, dtype=np.int64)
    d2 = sq_dist(q, feats[rows])
    order = np.lexsort((rows, d2))
    rows, d2 = rows[order], d2[order]
    idx = np.full(k, -1, dtype=np.int64)
    dist = np.full(k, np.inf)
    m = min(k, len(rows))
    idx[:m], dist[:m] = rows[:m], d2[:m]
    if len(rows) > k:
        gap = _rel_gap(d2[k - 1], d2[k])
    else:
        gap = math.inf
    if m == 0:
        band = (np.zeros(0, np.int64), np.zeros(0))
    else:
        dk = d2[m - 1]
        sel = np.abs(d2 - dk) <= tie_rel * dk
        band = (rows[sel], d2[sel])
    return idx, dist, gap, band


def retrieve(feats, region_of, n_regions_total, q, k, n_reg, reps=None, regions=None):
    """Two-stage retrieval of every query row of q.

    feats: n x d (float32 or float64); region_of: n ints in [0, R);
    reps: optional R x d representatives (default: region means);
    regions: optional per-query lists of region ids to search instead of the
    coarse selection (used to judge a frame on another selection of regions).

    Returns a dict of per-query arrays: regions (list of id arrays), region_d2,
    gap_r, idx (nq x k), d2 (nq x k, FP64), gap_k, n_cand, band (list).
    """
    # the rows keep their stored type: sq_dist promotes the gathered rows to
    # FP64 (exact for float32), so a large database is never copied whole
    f = np.asarray(feats)
    reg = np.asarray(region_of, dtype=np.int64)
    qs = np.atleast_2d(np.asarray(q, dtype=np.float64))
    if reps is None:
        reps64, nonempty = region_means(f, reg, n_regions_total)
    else:
        reps64 = np.asarray(reps, dtype=np.float64)
        nonempty = np.bincount(reg, minlength=n_regions_total) > 0
    order = np.argsort(reg, kind="stable")
    starts = np.zeros(n_regions_total + 1, dtype=np.int64)
    np.cumsum(np.bincount(reg, minlength=n_regions_total), out=starts[1:])
    nq = qs.shape[0]
    out = dict(regions=[], region_d2=[], gap_r=np.zeros(nq), idx=np.zeros((nq, k), np.int64),
               d2=np.zeros((nq, k)), gap_k=np.zeros(nq), n_cand=np.zeros(nq, np.int64), band=[])
    for i in range(nq):
        if regions is None:
            ids, rd2, gr = select_regions(qs[i], reps64, nonempty, n_reg)
        else:
            ids = np.asarray(regions[i], dtype=np.int64)
            rd2, gr = sq_dist(qs[i], reps64[ids]), math.nan
        rows = np.concatenate([order[starts[r]:starts[r + 1]] for r in ids]) if len(ids) else \
            np.zeros(0, np.int64)
        idx, dist, gk, band = search_rows(qs[i], f, rows, k)
        out["regions"].append(ids)
        out["region_d2"].append(rd2)
        out["gap_r"][i] = gr
        out["idx"][i], out["d2"][i], out["gap_k"][i] = idx, dist, gk
        out["n_cand"][i] = len(rows)
        out["band"].append(band)
    return out


def tile_of(xy: np.ndarray, cell: float) -> np.ndarray:
    """Integer tile (ix, iy) = (floor(x / cell), floor(y / cell)) of each
    position, origin (0, 0); x grows west to east, y south to north."""
    xy = np.asarray(xy, dtype=np.float64)
    return np.floor(xy / cell).astype(np.int64)


def aggregate(cand_rows, xy, cell, top_c, radius, toler_pct):
    """Algorithm 2 for one request.

    cand_rows: database row indices of the pooled candidates (duplicates count,
    -1 is padding and is dropped). Returns (ix, iy, x, y, flag).
    """
    rows = np.asarray(cand_rows, dtype=np.int64)
    rows = rows[rows >= 0]
    if len(rows) == 0:
        return 0, 0, math.nan, math.nan, FLAG_EMPTY
    t = tile_of(np.asarray(xy)[rows], cell)
    counts = {}
    for ix, iy in t.tolist():
        counts[(ix, iy)] = counts.get((ix, iy), 0) + 1
    total = len(rows)
    ranked = sorted(counts.items(), key=lambda kv: (-kv[1], kv[0][1], kv[0][0]))
    rho = int(math.floor(radius / cell + 0.5))
    chosen, flag = ranked[0][0], FLAG_LOW_CONFIDENCE
    for (tx, ty), _ in ranked[:top_c]:
        circle = sum(c for (ux, uy), c in counts.items()
                     if (ux - tx) ** 2 + (uy - ty) ** 2 <= rho * rho)
        if 100 * circle > toler_pct * total:
            chosen, flag = (tx, ty), 0
            break
    ix, iy = chosen
    return ix, iy, (ix + 0.5) * cell, (iy + 0.5) * cell, flag


def localize(feats, xy, region_of, n_regions_total, q, req_offsets, k, n_reg, agg, reps=None,
             regions=None, req_frames=None):
    """Whole path: retrieve every frame, pool each request's frames, aggregate.

    agg = (cell_m, top_c, radius_m, toler_pct). Returns the retrieve() dict
    plus per-request arrays tile (nreq x 2), pos (nreq x 2) and flags.
    Request i pools frames req_offsets[i] .. req_offsets[i+1]-1, or, with
    req_frames, the frames req_frames[req_offsets[i] : req_offsets[i+1]]
    (indices into q, in that order, repeats pooled again): the sliding
    window of Section 3.1, where consecutive requests share all but one
    frame and each frame is retrieved once.
    """
    res = retrieve(feats, region_of, n_regions_total, q, k, n_reg, reps=reps, regions=regions)
    offs = np.asarray(req_offsets, dtype=np.int64)
    nreq = len(offs) - 1
    tile = np.zeros((nreq, 2), np.int64)
    pos = np.zeros((nreq, 2))
    flags = np.zeros(nreq, np.int32)
    for i in range(nreq):
        if req_frames is None:
            frames = np.arange(offs[i], offs[i + 1])
        else:
            frames = np.asarray(req_frames, dtype=np.int64)[offs[i]:offs[i + 1]]
        pooled = res["idx"][frames].ravel()
        ix, iy, x, y, fl = aggregate(pooled, xy, *agg)
        tile[i], pos[i], flags[i] = (ix, iy), (x, y), fl
    res.update(tile=tile, pos=pos, flags=flags)
    return res


# ------------------------------------------------- per-subspace top-N
def localize_labels(feats, xy, region_of, n_regions_total, labels, q, req_offsets, k, n_reg,
                    agg):
    """Top-N per (frame, subspace) (Section 4 keeps N candidates per walked
    path: N x M x P of them for a request of M frames over P paths).

    labels: one subspace label per region, in [0, P). For every label p each
    frame runs the two-stage search restricted to the regions labelled p (the
    best n_reg of them by (d^2 to the mean, id), then their rows); request i
    pools, for each of its frames and each label, that frame's k results, and
    is aggregated as in localize. Returns idx / d2 as P x nq x k, per label
    the per-frame lists of retrieve (regions, gap_r, gap_k, band) under
    "per_label", and the per-request tile, pos and flags.
    """
    f = np.asarray(feats)
    qs = np.atleast_2d(np.asarray(q, dtype=np.float64))
    lab = np.asarray(labels, dtype=np.int64)
    P = int(lab.max()) + 1 if len(lab) else 0
    reps, nonempty = region_means(f, region_of, n_regions_total)
    idx = np.full((P, len(qs), k), -1, dtype=np.int64)
    d2 = np.full((P, len(qs), k), np.inf)
    per_label = []
    for p in range(P):
        keep = nonempty & (lab == p)
        if not keep.any():
            per_label.append(None)
            continue
        sel = [select_regions(qi, reps, keep, n_reg) for qi in qs]
        res = retrieve(f, region_of, n_regions_total, qs, k, n_reg, regions=[s_[0] for s_ in sel])
        # the coarse gap is the one of the label's own region ranking
        res["gap_r"] = np.array([s_[2] for s_ in sel])
        idx[p], d2[p] = res["idx"], res["d2"]
        per_label.append(res)
    offs = np.asarray(req_offsets, dtype=np.int64)
    nreq = len(offs) - 1
    tile = np.zeros((nreq, 2), np.int64)
    pos = np.zeros((nreq, 2))
    flags = np.zeros(nreq, np.int32)
    for i in range(nreq):
        pooled = idx[:, offs[i]:offs[i + 1]].transpose(1, 0, 2).ravel()
        ix, iy, x, y, fl = aggregate(pooled, xy, *agg)
        tile[i], pos[i], flags[i] = (ix, iy), (x, y), fl
    return dict(idx=idx, d2=d2, tile=tile, pos=pos, flags=flags, per_label=per_label)


# ------------------------------------------------- omnidirectional feature
def fft_magnitude(signals, d: int) -> np.ndarray:
    """Rotation-invariant omnidirectional feature (Section 3): the magnitude
    of the discrete Fourier transform of a 1-D panoramic signal.

    For each row x of `signals` (m x L, L >= 2) returns
        |X_j| = | sum_{t < L} x_t exp(-2 pi i j t / L) |,  j = 0 .. d-1,
    with 1 <= d <= L/2 + 1 (the remaining bins mirror these for real x).
    Written out from the definition in FP64, with no fast transform: the
    angle of each term is reduced exactly (j t mod L) before the cosine and
    sine, the two real sums are a plain matrix product, and the magnitude is
    sqrt(re^2 + im^2). A circular shift of x (a rotation of the panorama)
    multiplies X_j by a unit phase and leaves |X_j| unchanged.
    """
    x = np.asarray(signals, dtype=np.float64)
    if x.ndim != 2 or x.shape[1] < 2:
        raise ValueError("signals must be m x L with L >= 2")
    L = x.shape[1]
    if not 1 <= d <= L // 2 + 1:
        raise ValueError(f"d must be in 1..{L // 2 + 1}")
    j = np.arange(d, dtype=np.int64)[:, None]
    t = np.arange(L, dtype=np.int64)[None, :]
    angle = (2.0 * math.pi / L) * ((j * t) % L)
    re = x @ np.cos(angle).T
    im = -(x @ np.sin(angle).T)
    return np.sqrt(re * re + im * im)
