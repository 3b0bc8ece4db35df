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

// Per frame: offset of each kept region in the frame's candidate list, and the
// list length. Per region: how many frames kept it.
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

// One block: exclusive scans over regions of the frame counts (-> rq_off) and
// of the work-item counts (-> item_off, n_items); clears rfill.
__global__ __launch_bounds__(1024) void k_sched_scan(const int32_t *__restrict__ rcount, int R,
                                                     const int64_t *__restrict__ reg_start, int T,
                                                     int32_t *rq_off, int32_t *item_off,
                                                     int32_t *n_items, int32_t *rfill) {
  __shared__ int s_a[1024], s_b[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (R + nt - 1) / nt;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  int sa = 0, sb = 0;
  for (int r = r0; r < r1; ++r) {
    const int g = rcount[r];
    const int64_t rows = reg_start[r + 1] - reg_start[r];
    sa += g;
    if (g > 0) sb += (int)((rows + T - 1) / T) * ((g + kGroup - 1) / kGroup);
  }
  s_a[tid] = sa;
  s_b[tid] = sb;
  __syncthreads();
  // Hillis-Steele inclusive scan over the per-thread sums
  for (int o = 1; o < nt; o <<= 1) {
    const int va = tid >= o ? s_a[tid - o] : 0;
    const int vb = tid >= o ? s_b[tid - o] : 0;
    __syncthreads();
    s_a[tid] += va;
    s_b[tid] += vb;
    __syncthreads();
  }
  int ba = s_a[tid] - sa, bb = s_b[tid] - sb;
  for (int r = r0; r < r1; ++r) {
    const int g = rcount[r];
    const int64_t rows = reg_start[r + 1] - reg_start[r];
    rq_off[r] = ba;
    item_off[r] = bb;
    rfill[r] = 0;
    ba += g;
    if (g > 0) bb += (int)((rows + T - 1) / T) * ((g + kGroup - 1) / kGroup);
  }
  if (tid == nt - 1) n_items[0] = s_b[nt - 1];
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

__global__ void k_sched_items(int R, const int32_t *__restrict__ rcount,
                              const int32_t *__restrict__ item_off,
                              const int32_t *__restrict__ rq_off,
                              const int64_t *__restrict__ reg_start, int T, Item *items) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int g = rcount[r];
  if (g == 0) return;
  const int rows = (int)(reg_start[r + 1] - reg_start[r]);
  const int nch = (rows + T - 1) / T, ngr = (g + kGroup - 1) / kGroup;
  int o = item_off[r];
  for (int c = 0; c < nch; ++c)
    for (int b = 0; b < ngr; ++b) {
      Item it;
      it.row_begin = (int32_t)reg_start[r] + c * T;
      it.chunk_row = c * T;
      it.q0 = rq_off[r] + b * kGroup;
      it.nrows_gq = (min(T, rows - c * T) << 16) | min(kGroup, g - b * kGroup);
      items[o++] = it;
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

// The whole schedule in one block, for batches of up to kFusedPairs
// (frame, region) pairs: the same five steps with barriers in between.
constexpr int64_t kFusedPairs = 65536;

__device__ __forceinline__ int items_of(int g, int64_t rows, int T) {
  return g > 0 ? (int)((rows + T - 1) / T) * ((g + kGroup - 1) / kGroup) : 0;
}

__global__ __launch_bounds__(1024) void k_sched_fused(const int32_t *__restrict__ regions, int nq,
                                                      int nr, int R,
                                                      const int64_t *__restrict__ reg_start, int T,
                                                      int32_t *rcount, int32_t *rfill,
                                                      int32_t *rq_off, int32_t *item_off,
                                                      int32_t *cand_off, int32_t *n_cand,
                                                      int32_t *n_items, int2 *rq, Item *items) {
  __shared__ int s_a[16], s_b[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int r = tid; r < R; r += nt) {
    rcount[r] = 0;
    rfill[r] = 0;
  }
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
      for (int u = 0; u < 8; ++u) sz[u] = r[u] >= 0 ? (int)(reg_start[r[u] + 1] - reg_start[r[u]]) : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (j0 + u >= nr) break;
        cand_off[(int64_t)f * nr + j0 + u] = off;
        off += sz[u];
        if (r[u] >= 0) atomicAdd(&rcount[r[u]], 1);
      }
    }
    n_cand[f] = off;
  }
  __syncthreads();
  const int per = (R + nt - 1) / nt;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  int sa = 0, sb = 0;
  for (int r = r0; r < r1; ++r) {
    const int g = __hip_atomic_load(&rcount[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sa += g;
    sb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  // inclusive scans of (sa, sb) over the block: shuffles within each wave,
  // then the wave totals
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
    const int g = __hip_atomic_load(&rcount[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    rq_off[r] = ba;
    item_off[r] = bb;
    ba += g;
    bb += items_of(g, reg_start[r + 1] - reg_start[r], T);
  }
  if (tid == nt - 1) n_items[0] = ib;
  __syncthreads();
  const int64_t pairs = (int64_t)nq * nr;
  for (int64_t t = tid; t < pairs; t += nt) {
    const int r = regions[t];
    if (r < 0 || r >= R) continue;
    const int pos = rq_off[r] + atomicAdd(&rfill[r], 1);
    rq[pos] = make_int2((int)(t / nr), cand_off[t]);
  }
  __syncthreads();
  for (int r = tid; r < R; r += nt) {
    const int g = __hip_atomic_load(&rcount[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (g == 0) continue;
    const int rows = (int)(reg_start[r + 1] - reg_start[r]);
    const int nch = (rows + T - 1) / T, ngr = (g + kGroup - 1) / kGroup;
    int o = item_off[r];
    for (int c = 0; c < nch; ++c)
      for (int b = 0; b < ngr; ++b) {
        Item it;
        it.row_begin = (int32_t)reg_start[r] + c * T;
        it.chunk_row = c * T;
        it.q0 = rq_off[r] + b * kGroup;
        it.nrows_gq = (min(T, rows - c * T) << 16) | min(kGroup, g - b * kGroup);
        items[o++] = it;
      }
  }
}

hipError_t launch_sched(const int32_t *regions, int32_t nq, int32_t nr, int32_t R,
                        const int64_t *reg_start, int32_t T, int32_t *rcount, int32_t *rfill,
                        int32_t *rq_off, int32_t *item_off, int32_t *cand_off, int32_t *n_cand,
                        int32_t *n_items, int2 *rq, Item *items, hipStream_t s) {
  if ((int64_t)nq * nr <= kFusedPairs) {
    return launch_kernel(k_sched_fused, dim3(1), dim3(1024), 0, s, regions, nq, nr, R, reg_start, T,
                       rcount, rfill, rq_off, item_off, cand_off, n_cand, n_items, rq, items);
  }
  hipError_t e = launch_fill_i32(rcount, R, 0, s);
  if (e != hipSuccess) return e;
  if (nq > 0) {
    if ((e = launch_kernel(k_sched_count, dim3((nq + 255) / 256), dim3(256), 0, s, regions, nq, nr,
                       R, reg_start, rcount, cand_off, n_cand)) != hipSuccess) return e;
  }
  if ((e = launch_kernel(k_sched_scan, dim3(1), dim3(1024), 0, s, rcount, R, reg_start, T, rq_off,
                     item_off, n_items, rfill)) != hipSuccess) return e;
  const int64_t pairs = (int64_t)nq * nr;
  if (pairs > 0) {
    if ((e = launch_kernel(k_sched_scatter, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s,
                       regions, nq, nr, R, cand_off, rq_off, rfill, rq)) != hipSuccess) return e;
  }
  return launch_kernel(k_sched_items, dim3((R + 255) / 256), dim3(256), 0, s, R, rcount, item_off,
                     rq_off, reg_start, T, items);
}

}  // namespace hloc
