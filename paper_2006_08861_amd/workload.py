"""Seeded synthetic workloads shaped like the paper's indoor-localization database.

The paper models one floor of a building along five parallel walked paths and
stores one omnidirectional feature per captured frame (Section 4); a query is a
short clip of frames taken near one spot (Section 3.1). The real capture is not
available, so this module draws stand-ins with the same structure:

* features: a stationary AR(1) random walk along the walked path (neighbouring
  frames look alike, as consecutive video frames do), L2-normalised, float32;
* positions: the walk runs at uniform arc length along a serpentine of five
  100 m corridors joined by 8 m connectors (a 100 x 40 m floor); larger
  databases tile further floors in the plane;
* regions: consecutive runs of the walk with equal, uniform or lognormal sizes;
* queries: a database frame plus Gaussian noise; multi-frame requests draw
  their frames within +-1 m of arc length of a centre frame, with a fraction
  replaced by decoys from another region (the paper's scene-similarity problem,
  Section 3).

* panoramic signals: 1-D omnidirectional signals (one grey level per viewing
  direction) for the Fourier-magnitude feature of Section 3.

Inputs only: nothing in this module computes a distance, a ranking, a tile or
a vote. Both the HIP path and the oracle receive what it returns.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.signal import lfilter

FLOOR_CORRIDOR_Y = (4.0, 12.0, 20.0, 28.0, 36.0)
FLOOR_LENGTH_X = 100.0
CONNECTOR_M = 8.0
PATH_LENGTH_M = len(FLOOR_CORRIDOR_Y) * FLOOR_LENGTH_X + (len(FLOOR_CORRIDOR_Y) - 1) * CONNECTOR_M
ENTRIES_PER_FLOOR = 10_000
FLOOR_TILE_DX, FLOOR_TILE_DY, FLOORS_PER_ROW = 120.0, 60.0, 16
WALK_STEP = 0.05


def _path_point(s: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(x, y) of arc length s (metres) along the serpentine of one floor."""
    seg = FLOOR_LENGTH_X + CONNECTOR_M
    leg = np.minimum((s // seg).astype(np.int64), len(FLOOR_CORRIDOR_Y) - 1)
    t = s - leg * seg
    y0 = np.asarray(FLOOR_CORRIDOR_Y)[leg]
    on_corr = t <= FLOOR_LENGTH_X
    fwd = (leg % 2) == 0
    xc = np.where(fwd, t, FLOOR_LENGTH_X - t)
    xe = np.where(fwd, FLOOR_LENGTH_X, 0.0)
    x = np.where(on_corr, xc, xe)
    y = np.where(on_corr, y0, y0 + (t - FLOOR_LENGTH_X))
    return x, y


def corridor_xy(n: int) -> np.ndarray:
    """Floor-plan position (metres, float64, n x 2) of each of n walk entries."""
    i = np.arange(n, dtype=np.int64)
    floor = i // ENTRIES_PER_FLOOR
    s = (i % ENTRIES_PER_FLOOR) * (PATH_LENGTH_M / ENTRIES_PER_FLOOR)
    x, y = _path_point(s)
    xy = np.empty((n, 2), dtype=np.float64)
    xy[:, 0] = x + (floor % FLOORS_PER_ROW) * FLOOR_TILE_DX
    xy[:, 1] = y + (floor // FLOORS_PER_ROW) * FLOOR_TILE_DY
    return xy


def walk_features(n: int, d: int, rng: np.random.Generator, step: float = WALK_STEP,
                  block: int = 65536) -> np.ndarray:
    """n x d float32 features: stationary AR(1) walk x_t = rho x_{t-1} + s_t,
    s_t ~ N(0, step^2 I), rho = sqrt(1 - step^2) (unit per-dim variance), each
    row divided by its L2 norm."""
    rho = math.sqrt(1.0 - step * step)
    out = np.empty((n, d), dtype=np.float32)
    zi = np.zeros((1, d))
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        s = rng.standard_normal((b1 - b0, d)) * step
        if b0 == 0:
            s[0] = rng.standard_normal(d)
        # the recursion runs along rows; filtering the transposed block runs it
        # over contiguous memory (the same arithmetic, three times faster)
        yt, zt = lfilter([1.0], [1.0, -rho], np.ascontiguousarray(s.T), axis=1, zi=zi.T)
        y, zi = yt.T, zt.T
        y /= np.linalg.norm(y, axis=1, keepdims=True)
        out[b0:b1] = y
    return out


def rescale_sizes(sizes: np.ndarray, n: int) -> np.ndarray:
    """Integer sizes >= 1 proportional to `sizes` that sum to exactly n
    (largest-remainder rounding)."""
    sizes = np.asarray(sizes, dtype=np.float64)
    r = len(sizes)
    if n < r:
        raise ValueError("fewer entries than regions")
    want = sizes * (n / sizes.sum())
    base = np.maximum(np.floor(want).astype(np.int64), 1)
    rem = n - int(base.sum())
    if rem > 0:
        order = np.argsort(-(want - np.floor(want)), kind="stable")
        base[order[:rem]] += 1
    while rem < 0:
        order = np.argsort(-base, kind="stable")
        take = min(-rem, int((base[order] > 1).sum()))
        base[order[:take]] -= 1
        rem += take
    return base


def region_sizes(kind: str, n: int, r: int, rng: np.random.Generator,
                 lo: int = 50, hi: int = 400, sigma: float = 1.0) -> np.ndarray:
    """Sizes of r consecutive regions summing to n. Only the shape of the draw
    matters (equal, uniform in [lo, hi], lognormal of log-sd sigma): the draw is
    rescaled to sum to n."""
    if kind == "equal":
        raw = np.full(r, n / r)
    elif kind == "uniform":
        raw = rng.integers(lo, hi + 1, size=r).astype(np.float64)
    elif kind == "lognormal":
        raw = rng.lognormal(0.0, sigma, size=r)
    else:
        raise ValueError(kind)
    return rescale_sizes(raw, n)


def region_of_from_sizes(sizes: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)


@dataclasses.dataclass
class Workload:
    feats: np.ndarray          # n x d float32
    xy: np.ndarray             # n x 2 float64, metres
    region_of: np.ndarray      # n int32
    n_regions_total: int
    q: np.ndarray              # nq x d float32
    req_offsets: np.ndarray    # nreq + 1 int32
    truth: np.ndarray          # nreq int64, the database entry each request was drawn around
    k: int
    n_reg: int
    agg: tuple                 # (cell_m, top_c, radius_m, toler_pct)
    name: str = ""


def single_frame_queries(feats: np.ndarray, nq: int, sigma: float, rng: np.random.Generator):
    j = rng.integers(0, feats.shape[0], size=nq)
    q = feats[j].astype(np.float64) + rng.normal(0.0, sigma, size=(nq, feats.shape[1]))
    return q.astype(np.float32), j.astype(np.int64)


def multi_frame_requests(feats: np.ndarray, region_of: np.ndarray, n_req: int, frames,
                         sigma: float, decoy_p: float, window_m: float,
                         rng: np.random.Generator):
    """Requests of F frames each (F fixed, or drawn uniformly from a (lo, hi)
    pair). Frames sit within +-window_m of arc length of a centre entry on the
    same floor; each is replaced with probability decoy_p by an entry drawn from
    a different region. Every frame gets N(0, sigma^2) noise per dimension."""
    n, d = feats.shape
    spacing = PATH_LENGTH_M / ENTRIES_PER_FLOOR
    if isinstance(frames, tuple):
        f_per = rng.integers(frames[0], frames[1] + 1, size=n_req)
    else:
        f_per = np.full(n_req, int(frames))
    offs = np.zeros(n_req + 1, dtype=np.int64)
    np.cumsum(f_per, out=offs[1:])
    total = int(offs[-1])
    centre = rng.integers(0, n, size=n_req)
    rows = np.empty(total, dtype=np.int64)
    for i in range(n_req):
        c = int(centre[i])
        fl0 = (c // ENTRIES_PER_FLOOR) * ENTRIES_PER_FLOOR
        fl1 = min(n, fl0 + ENTRIES_PER_FLOOR) - 1
        u = rng.uniform(-window_m, window_m, size=int(f_per[i]))
        j = np.clip(c + np.rint(u / spacing).astype(np.int64), fl0, fl1)
        decoy = rng.random(int(f_per[i])) < decoy_p
        if region_of.min() == region_of.max():
            decoy[:] = False
        for t in np.nonzero(decoy)[0]:
            while True:
                cand = int(rng.integers(0, n))
                if region_of[cand] != region_of[j[t]]:
                    j[t] = cand
                    break
        rows[offs[i]:offs[i + 1]] = j
    q = feats[rows].astype(np.float64) + rng.normal(0.0, sigma, size=(total, d))
    return q.astype(np.float32), offs.astype(np.int32), centre.astype(np.int64)


# Workload shapes. Index i uses seed 1000 + i; a shape with db=j queries the
# database of shape j (drawn with seed 1000 + j): the multi-frame shape runs on
# the same 2M x 512 database as the precision shape. Aggregation tuples are
# (cell_m, top_c, radius_m, toler_pct): single-frame shapes take the argmax of
# a 0.5 m grid vote, multi-frame shapes the paper's 0.30 m tiles, ten top
# tiles, 3 m tolerance circle and 20 % (Section 3.2).
ARGMAX_05 = (0.5, 1, 0.0, 0)
PAPER_AGG = (0.30, 10, 3.0, 20)
SHAPES = [
    dict(name="cpu-10k-d256", n=10_000, d=256, r=50, sizes="equal", nq=1000, frames=1,
         n_reg=5, k=10, sigma=0.1, agg=ARGMAX_05),
    dict(name="fp32-200k-d256", n=200_000, d=256, r=1024, sizes="uniform", lo=50, hi=400,
         nq=256, frames=1, n_reg=8, k=16, sigma=0.1, agg=ARGMAX_05),
    dict(name="bf16-2m-d512", n=2_000_000, d=512, r=4096, sizes="lognormal",
         nq=2048, frames=1, n_reg=8, k=16, sigma=0.1, agg=ARGMAX_05),
    dict(name="fp8-2m-d512-8frame", n=2_000_000, d=512, r=4096, sizes="lognormal",
         nq=4096, frames=8, n_reg=8, k=32, sigma=0.15, agg=PAPER_AGG, db=2),
    dict(name="serve-4m-d256", n=4_000_000, d=256, r=16384, sizes="lognormal",
         nq=4096, frames=(1, 16), n_reg=8, k=32, sigma=0.15, agg=PAPER_AGG),
]


def make_database(n: int, d: int, r: int, sizes: str, seed: int, lo: int = 50, hi: int = 400):
    rng = np.random.default_rng(seed)
    feats = walk_features(n, d, rng)
    xy = corridor_xy(n)
    sz = region_sizes(sizes, n, r, rng, lo=lo, hi=hi)
    return feats, xy, region_of_from_sizes(sz)


def make_workload(index: int, nq: int | None = None, n: int | None = None,
                  r: int | None = None, seed: int | None = None, database=None) -> Workload:
    """Workload `index` of SHAPES. nq, n and r override the batch size, the
    database size and the region count (small parity cases of the same shape;
    r defaults to keeping the mean region size); seed replaces both the
    database's and the queries' seed. database = (feats, xy, region_of) of an
    earlier workload of the same database (same shape of rows and regions)
    skips drawing it again."""
    s = dict(SHAPES[index])
    db_seed = 1000 + s.get("db", index) if seed is None else seed
    seed = 1000 + index if seed is None else seed
    if n is not None:
        r = r if r is not None else max(1, round(s["r"] * n / s["n"]))
        s["n"] = n
    if r is not None:
        s["r"] = r
    if database is not None:
        feats, xy, region_of = database
        if feats.shape != (s["n"], s["d"]) or int(region_of.max()) >= s["r"]:
            raise ValueError("the database given does not have this workload's shape")
    else:
        feats, xy, region_of = make_database(s["n"], s["d"], s["r"], s["sizes"], db_seed,
                                             lo=s.get("lo", 50), hi=s.get("hi", 400))
    rng = np.random.default_rng(seed + 7)
    count = s["nq"] if nq is None else nq
    if s["frames"] == 1:
        q, truth = single_frame_queries(feats, count, s["sigma"], rng)
        offs = np.arange(count + 1, dtype=np.int32)
    else:
        q, offs, truth = multi_frame_requests(feats, region_of, count, s["frames"], s["sigma"],
                                              0.10, 1.0, rng)
    return Workload(feats, xy, region_of, int(s["r"]), q, offs, truth, s["k"], s["n_reg"],
                    s["agg"], s["name"])


def panoramic_signals(n: int, length: int, rng: np.random.Generator) -> np.ndarray:
    """Stand-ins for 1-D omnidirectional signals, float32 n x length (one value
    per viewing direction around the camera, such as a column mean of the
    panorama): a grey level of 128, a smooth periodic profile (white noise
    circularly smoothed by a Gaussian of width length / 32, centred and scaled
    to standard deviation 40) and pixel noise of standard deviation 2."""
    if length < 2:
        raise ValueError("length must be >= 2")
    w = max(1.0, length / 32)
    half = int(min(length // 2, math.ceil(3 * w)))
    taps = np.exp(-0.5 * (np.arange(-half, half + 1) / w) ** 2)
    white = rng.standard_normal((n, length))
    padded = np.concatenate([white[:, length - half:], white, white[:, :half]], axis=1)
    smooth = lfilter(taps, [1.0], padded, axis=1)[:, 2 * half:]
    smooth -= smooth.mean(axis=1, keepdims=True)
    smooth *= 40.0 / np.maximum(smooth.std(axis=1, keepdims=True), 1e-12)
    return (128.0 + smooth + 2.0 * rng.standard_normal((n, length))).astype(np.float32)
