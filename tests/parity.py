"""Acceptance rule for comparing the HIP path with the FP64 oracle.

Per frame:
  * regions: the GPU's region set must equal the oracle's unless the oracle's
    relative gap between the n-th and (n+1)-th region is below TIE; such a frame
    is then judged on the GPU's own regions (region-tie excused);
  * indices: if the oracle's relative gap between the k-th and (k+1)-th
    distance is at least TIE, the GPU's index set must equal the oracle's;
    otherwise the rows strictly inside (d < d_k (1 - TIE)) must match and the
    rest must come from the oracle's tie band;
  * order: positions whose oracle distance is separated from both neighbours
    by at least TIE must hold the oracle's index;
  * distances: |d_gpu - d_ora| <= DIST_RTOL * d_ora rank by rank, and exactly
    0 where the oracle's distance is 0; padding (-1, +inf) must coincide.
Per request: the estimate (tile, flag, xy) must equal, bit for bit, the
oracle's aggregation of the GPU's own pooled candidates, and the oracle's
end-to-end estimate whenever the pooled candidate multisets agree.
"""
import math

import numpy as np

import oracle

TIE = 1e-6
DIST_RTOL = 1e-5


def judge_frames(gpu_idx, gpu_dist, gpu_regions, ora, feats, region_of, R, q, k, reps=None):
    gpu_idx = np.asarray(gpu_idx)
    gpu_dist = np.asarray(gpu_dist, dtype=np.float64)
    st = dict(frames=len(gpu_idx), region_excused=0, tie_excused=0, hits=0, total=0,
              max_rel_err=0.0, exact_lists=0)
    for i in range(len(gpu_idx)):
        o_idx, o_d2, gap_k = ora["idx"][i], ora["d2"][i], ora["gap_k"][i]
        band = ora["band"][i]
        if gpu_regions is not None:
            gr = set(np.asarray(gpu_regions[i]).tolist())
            orr = set(np.asarray(ora["regions"][i]).tolist())
            if gr != orr:
                assert ora["gap_r"][i] < TIE, \
                    f"frame {i}: regions {sorted(gr)} vs oracle {sorted(orr)} (gap {ora['gap_r'][i]})"
                sub = oracle.retrieve(feats, region_of, R, q[i:i + 1], k, len(gr), reps=reps,
                                      regions=[np.asarray(gpu_regions[i])])
                o_idx, o_d2, gap_k, band = sub["idx"][0], sub["d2"][0], sub["gap_k"][0], sub["band"][0]
                st["region_excused"] += 1
        g_idx, g_d = gpu_idx[i], gpu_dist[i]
        valid = o_idx >= 0
        assert np.array_equal(g_idx >= 0, valid), f"frame {i}: padding differs {g_idx} vs {o_idx}"
        assert np.all(np.isinf(g_d[~valid])), f"frame {i}: padding distance not +inf"
        m = int(valid.sum())
        gs, os_ = set(g_idx[:m].tolist()), set(o_idx[:m].tolist())
        if gap_k >= TIE:
            assert gs == os_, f"frame {i}: index set differs (gap {gap_k}): {g_idx} vs {o_idx}"
        else:
            dk = o_d2[m - 1]
            inner = set(o_idx[:m][o_d2[:m] < dk * (1 - TIE)].tolist())
            assert inner <= gs, f"frame {i}: rows inside the tie band missing"
            assert gs - inner <= set(band[0].tolist()), f"frame {i}: rows outside the tie band"
            if gs != os_:
                st["tie_excused"] += 1
        for j in range(m):
            lo = j == 0 or (o_d2[j] - o_d2[j - 1]) >= TIE * o_d2[j]
            hi = j == m - 1 or (o_d2[j + 1] - o_d2[j]) >= TIE * o_d2[j + 1]
            if lo and hi and (j < m - 1 or gap_k >= TIE):
                assert g_idx[j] == o_idx[j], f"frame {i} rank {j}: {g_idx[j]} vs {o_idx[j]}"
        zero = o_d2[:m] == 0
        assert np.all(g_d[:m][zero] == 0), f"frame {i}: exact match not at distance 0"
        err = np.abs(g_d[:m] - o_d2[:m])
        assert np.all(err <= DIST_RTOL * o_d2[:m]), f"frame {i}: distance error {err.max()}"
        if m:
            rel = err[~zero] / o_d2[:m][~zero]
            st["max_rel_err"] = max(st["max_rel_err"], float(rel.max()) if rel.size else 0.0)
        st["hits"] += len(gs & os_)
        st["total"] += m
        st["exact_lists"] += int(np.array_equal(g_idx, ora["idx"][i]))
    st["recall"] = st["hits"] / max(st["total"], 1)
    return st


def judge_requests(gpu_idx, gpu_xy, gpu_tile, gpu_flags, ora, xy, req_offsets, agg):
    """Aggregation parity; returns the number of requests whose pooled
    candidates equal the oracle's."""
    offs = np.asarray(req_offsets)
    same = 0
    for r in range(len(offs) - 1):
        pooled = np.asarray(gpu_idx[offs[r]:offs[r + 1]]).ravel()
        ix, iy, x, y, fl = oracle.aggregate(pooled, xy, *agg)
        assert [int(gpu_tile[r][0]), int(gpu_tile[r][1])] == [ix, iy], f"request {r}: tile"
        assert int(gpu_flags[r]) == fl, f"request {r}: flag {gpu_flags[r]} vs {fl}"
        for a, b in ((gpu_xy[r][0], x), (gpu_xy[r][1], y)):
            assert (math.isnan(a) and math.isnan(b)) or a == b, f"request {r}: xy {a} vs {b}"
        o_pooled = ora["idx"][offs[r]:offs[r + 1]].ravel()
        if sorted(pooled.tolist()) == sorted(o_pooled.tolist()):
            same += 1
            assert [ix, iy] == ora["tile"][r].tolist() and fl == ora["flags"][r]
            ox, oy = ora["pos"][r]
            assert (math.isnan(x) and math.isnan(ox)) or (x == ox and y == oy)
    return same
