// Scheduling of the fine screen: the frame -> regions lists chosen by the
// coarse stage are inverted into region -> frames lists, and every touched
// region is cut into chunks of T rows crossed with groups of up to 16 frames.
// This takes the place of the paper's one-stream-per-subspace launch
// (Section 3.1): a region's rows are read once per group of frames that kept
// it, and uneven regions become many equal-sized work items for one
// persistent kernel. Every count lives in device memory; no host round trip.
#include "hloc_device.h"
#include "hloc_internal.h"

#include <algorithm>

namespace hloc {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  return launch_kernel(k_fill_i32, dim3(grid), dim3(256), 0, s, p, n, v);
}

// Region owning work item t: the last r with item_off[r] <= t, for
// non-decreasing item_off with item_off[0] = 0 <= t < item_off[R]; that region
// has at least one item (item_off[r + 1] > t).
__device__ __forceinline__ int owner_region(const int32_t *item_off, int R, int t) {
  int lo = 0, hi = R;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item_off[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int items_of(int g, int64_t rows, int T) {
  return g > 0 ? (int)((rows + T - 1) / T) * ((g + kGroup - 1) / kGroup) : 0;
}

// Work item t of region r, whose frames are rq[q_begin, q_end): chunk-major,
// frame groups inner, so consecutive items re-read the same rows.
__device__ __forceinline__ Item make_item(int t, int r, int item_begin, int q_begin, int q_end,
                                          const int64_t *__restrict__ reg_start, int T) {
  const int g = q_end - q_begin, ngr = (g + kGroup - 1) / kGroup;
  const int local = t - item_begin, c = local / ngr, b = local - c * ngr;
  const int64_t r0 = reg_start[r];
  const int rows = (int)(reg_start[r + 1] - r0);
  Item it;
  it.row_begin = (int32_t)r0 + c * T;
  it.chunk_row = c * T;
  it.q0 = q_begin + b * kGroup;
  it.nrows_gq = (min(T, rows - c * T) << 16) | min(kGroup, g - b * kGroup);
  return it;
}

// Multi-kernel schedule for large region counts. Per frame: offset of each
// kept region in the frame's candidate list, and the list length. Per region:
// how many frames kept it.
__global__ void k_sched_count(const int32_t *__restrict__ regions, int nq, int nr, int R,
                              const int64_t *__restrict__ reg_start, int32_t *rcount,
                              int32_t *cand_off, int32_t *n_cand) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nq) return;
  int off = 0;
  for (int j = 0; j < nr; ++j) {
    const int r = regions[(int64_t)f * nr + j];
    cand_off[(int64_t)f * nr + j] = off;
    if (r < 0 || r >= R) continue;
    off += (int)(reg_start[r + 1] - reg_start[r]);
    atomicAdd(&rcount[r], 1);
  }
  n_cand[f] = off;
}

// One block: exclusive scans over regions of the frame counts (-> rq_off,
// R + 1 entries) and of the work-item counts (-> item_off, R + 1 entries);
// clears rfill.
__global__ __launch_bounds__(1024) void k_sched_scan(const int32_t *__restrict__ rcount, int R,
                                                     const int64_t *__restrict__ reg_start, int T,
                                                     int32_t *rq_off, int32_t *item_off,
                                                     int32_t *n_items, int32_t *rfill) {
  __shared__ int s_a[16], s_b[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (R + nt - 1) / nt;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  int sa = 0, sb = 0;
  for (int r = r0; r < r1; ++r) {
    const int g = rcount[r];
    sa += g;
    sb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  const int lane = tid & 63, wv = tid >> 6;
  int ia = sa, ib = sb;
  for (int o = 1; o < 64; o <<= 1) {
    const int ya = __shfl_up(ia, o), yb = __shfl_up(ib, o);
    if (lane >= o) {
      ia += ya;
      ib += yb;
    }
  }
  if (lane == 63) {
    s_a[wv] = ia;
    s_b[wv] = ib;
  }
  __syncthreads();
  for (int i = 0; i < wv; ++i) {
    ia += s_a[i];
    ib += s_b[i];
  }
  int ba = ia - sa, bb = ib - sb;
  for (int r = r0; r < r1; ++r) {
    const int g = rcount[r];
    rq_off[r] = ba;
    item_off[r] = bb;
    rfill[r] = 0;
    ba += g;
    bb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  if (tid == nt - 1) {
    rq_off[R] = ia;
    item_off[R] = ib;
    n_items[0] = ib;
  }
}

__global__ void k_sched_scatter(const int32_t *__restrict__ regions, int nq, int nr, int R,
                                const int32_t *__restrict__ cand_off,
                                const int32_t *__restrict__ rq_off, int32_t *rfill, int2 *rq) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nq * nr) return;
  const int f = (int)(t / nr);
  const int r = regions[t];
  if (r < 0 || r >= R) return;
  const int pos = rq_off[r] + atomicAdd(&rfill[r], 1);
  rq[pos] = make_int2(f, cand_off[t]);
}

// One thread per work item (grid-stride), each finding its region by binary
// search, so that a region kept by many frames is expanded by many threads.
__global__ void k_sched_items(int R, const int32_t *__restrict__ item_off,
                              const int32_t *__restrict__ rq_off,
                              const int64_t *__restrict__ reg_start, int T, Item *items) {
  const int n = item_off[R];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int r = owner_region(item_off, R, t);
    items[t] = make_item(t, r, item_off[r], rq_off[r], rq_off[r + 1], reg_start, T);
  }
}

// Exhaustive search (every non-empty region kept, the paper's whole-database
// search): every frame gets the same region list.
__global__ void k_broadcast_ids(const int32_t *__restrict__ ids, int nr, int64_t total,
                                int32_t *__restrict__ regions) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    regions[t] = ids[t % nr];
}

hipError_t launch_broadcast_ids(const int32_t *ids, int32_t nr, int32_t nq, int32_t *regions,
                                hipStream_t s) {
  const int64_t total = (int64_t)nr * nq;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  return launch_kernel(k_broadcast_ids, dim3(grid), dim3(256), 0, s, ids, nr, total, regions);
}

// The whole schedule in one block for up to kFusedMaxR regions and
// kFusedMaxPairs (frame, region) pairs: per-region
// counts, fill pointers and item offsets live in LDS, so the histogram and the
// scatter use LDS atomics (no contention on global memory when many frames
// keep the same region), and work items are expanded one per thread.
constexpr int kFusedMaxR = 16384;
constexpr int64_t kFusedMaxPairs = 8192;  // larger batches: the multi-kernel path is faster

size_t fused_lds_bytes(int R) { return (size_t)(2 * R + 1) * sizeof(int); }

__global__ __launch_bounds__(1024) void k_sched_fused(const int32_t *__restrict__ regions, int nq,
                                                      int nr, int R,
                                                      const int64_t *__restrict__ reg_start, int T,
                                                      int32_t *rq_off, int32_t *cand_off,
                                                      int32_t *n_cand, int32_t *n_items, int2 *rq,
                                                      Item *items) {
  extern __shared__ int s_mem[];
  int *s_fill = s_mem;     // R: frame counts, then fill pointers
  int *s_iof = s_mem + R;  // R + 1: item offsets
  __shared__ int s_a[16], s_b[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int r = tid; r < R; r += nt) s_fill[r] = 0;
  __syncthreads();
  for (int f = tid; f < nq; f += nt) {
    int off = 0;
    for (int j0 = 0; j0 < nr; j0 += 8) {
      // ids, then sizes, then updates: eight loads in flight per step
      int r[8], sz[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        r[u] = j0 + u < nr ? regions[(int64_t)f * nr + j0 + u] : -1;
        if (r[u] >= R) r[u] = -1;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        sz[u] = r[u] >= 0 ? (int)(reg_start[r[u] + 1] - reg_start[r[u]]) : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (j0 + u >= nr) break;
        cand_off[(int64_t)f * nr + j0 + u] = off;
        off += sz[u];
        if (r[u] >= 0) atomicAdd(&s_fill[r[u]], 1);
      }
    }
    n_cand[f] = off;
  }
  __syncthreads();
  // exclusive scans of (frames, items) over regions: a contiguous range of
  // regions per thread, shuffles within each wave, then the wave totals
  const int per = (R + nt - 1) / nt;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  int sa = 0, sb = 0;
  for (int r = r0; r < r1; ++r) {
    const int g = s_fill[r];
    sa += g;
    sb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  const int lane = tid & 63, wv = tid >> 6;
  int ia = sa, ib = sb;
  for (int o = 1; o < 64; o <<= 1) {
    const int ya = __shfl_up(ia, o), yb = __shfl_up(ib, o);
    if (lane >= o) {
      ia += ya;
      ib += yb;
    }
  }
  if (lane == 63) {
    s_a[wv] = ia;
    s_b[wv] = ib;
  }
  __syncthreads();
  for (int i = 0; i < wv; ++i) {
    ia += s_a[i];
    ib += s_b[i];
  }
  int ba = ia - sa, bb = ib - sb;
  for (int r = r0; r < r1; ++r) {
    const int g = s_fill[r];
    rq_off[r] = ba;
    s_fill[r] = ba;
    s_iof[r] = bb;
    ba += g;
    bb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  if (tid == nt - 1) {
    rq_off[R] = ia;
    s_iof[R] = ib;
    n_items[0] = ib;
  }
  __syncthreads();
  const int64_t pairs = (int64_t)nq * nr;
  for (int64_t t = tid; t < pairs; t += nt) {
    const int r = regions[t];
    if (r < 0 || r >= R) continue;
    const int pos = atomicAdd(&s_fill[r], 1);
    rq[pos] = make_int2((int)(t / nr), cand_off[t]);
  }
  __syncthreads();
  // after the scatter s_fill[r] is the end of region r's frames, which is
  // also where region r + 1's frames begin
  const int n = s_iof[R];
  for (int t = tid; t < n; t += nt) {
    const int r = owner_region(s_iof, R, t);
    items[t] = make_item(t, r, s_iof[r], r > 0 ? s_fill[r - 1] : 0, s_fill[r], reg_start, T);
  }
}

hipError_t prepare_sched_kernels() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sched_fused),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)fused_lds_bytes(kFusedMaxR));
}

hipError_t launch_sched(const int32_t *regions, int32_t nq, int32_t nr, int32_t R,
                        const int64_t *reg_start, int32_t T, int32_t *rcount, int32_t *rfill,
                        int32_t *rq_off, int32_t *item_off, int32_t *cand_off, int32_t *n_cand,
                        int32_t *n_items, int2 *rq, Item *items, hipStream_t s) {
  const int64_t pairs = (int64_t)nq * nr;
  if (R <= kFusedMaxR && pairs <= kFusedMaxPairs) {
    return launch_kernel(k_sched_fused, dim3(1), dim3(1024), (uint32_t)fused_lds_bytes(R), s,
                         regions, nq, nr, R, reg_start, T, rq_off, cand_off, n_cand, n_items, rq,
                         items);
  }
  hipError_t e = launch_fill_i32(rcount, R, 0, s);
  if (e != hipSuccess) return e;
  if (nq > 0) {
    if ((e = launch_kernel(k_sched_count, dim3((nq + 255) / 256), dim3(256), 0, s, regions, nq,
                           nr, R, reg_start, rcount, cand_off, n_cand)) != hipSuccess)
      return e;
  }
  if ((e = launch_kernel(k_sched_scan, dim3(1), dim3(1024), 0, s, rcount, R, reg_start, T,
                         rq_off, item_off, n_items, rfill)) != hipSuccess)
    return e;
  if (pairs > 0) {
    if ((e = launch_kernel(k_sched_scatter, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0,
                           s, regions, nq, nr, R, cand_off, rq_off, rfill, rq)) != hipSuccess)
      return e;
  }
  return launch_kernel(k_sched_items, dim3(1024), dim3(256), 0, s, R, item_off, rq_off, reg_start,
                       T, items);
}

}  // namespace hloc
