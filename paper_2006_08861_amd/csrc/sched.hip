// Scheduling of the fine screen: the frame -> regions lists chosen by the
// coarse stage are inverted into region -> frames lists, and every touched
// region is cut into chunks of T rows (for wide regions W rows, or a few runs
// of W rows) crossed with groups of up to kListFrames frames. This takes the place of the paper's
// one-stream-per-subspace launch (Section 3.1): uneven regions become many
// equal-sized work items for persistent screen kernels, and every count lives
// in device memory (no host round trip).
//
// Items come in two classes. A region kept by at most kGroup frames gives
// narrow items (one MFMA column block of frames); a region kept by more
// frames gives wide items of up to kListFrames frames, screened by a kernel
// that reads each row once for all of them. Narrow items are numbered first:
// items [0, n_items[4]) are narrow, [n_items[4], n_items[0]) wide. Regions
// are laid out in that order (narrow regions by id, then wide regions by id)
// in vord, with their first item in iof (non-decreasing), so the owner of an
// item is found by binary search.
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

// Slot owning work item t: the last k with iof[k] <= t, for non-decreasing
// iof with iof[0] = 0 <= t < iof[R]; that slot has at least one item.
__device__ __forceinline__ int owner_slot(const int32_t *iof, int R, int t) {
  int lo = 0, hi = R;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (iof[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Rows per chunk of a region kept by g frames: T for narrow regions, W (what
// the wide kernel of the screen takes) for wide ones. With WM > 1 a wide
// chunk is up to WM runs of W rows (the register-row kernels take such an
// item run by run with its frames staged once), as many as bring the item to
// about kWideSteps (W rows, kGroup frames) steps: items of few frame groups
// then carry enough work to hide their set-up.
__device__ __forceinline__ int chunk_rows(int g, int T, int W, int WM) {
  if (g <= kGroup) return T;
  const int groups = (min(g, kListFrames) + kGroup - 1) / kGroup;
  return W * max(1, min(WM, (kWideSteps + groups - 1) / groups));
}

__device__ __forceinline__ int items_of(int g, int64_t rows, int T, int W, int WM) {
  const int C = chunk_rows(g, T, W, WM);
  return g > 0 ? (int)((rows + C - 1) / C) * ((g + kListFrames - 1) / kListFrames) : 0;
}

// Work item t of a region whose rows are [r0, r0 + rows) and whose frames are
// rq[q_begin, q_end): chunk-major, frame groups inner, so consecutive items
// re-read the same rows.
__device__ __forceinline__ Item make_item(int t, int item_begin, int q_begin, int q_end, int r0,
                                          int rows, int T, int W, int WM) {
  const int g = q_end - q_begin, ngr = (g + kListFrames - 1) / kListFrames;
  const int C = chunk_rows(g, T, W, WM);
  const int local = t - item_begin, c = local / ngr, b = local - c * ngr;
  Item it;
  it.row_begin = r0 + c * C;
  it.chunk_row = c * C;
  it.q0 = q_begin + b * kListFrames;
  it.nrows_gq = (min(C, rows - c * C) << 16) | min(kListFrames, g - b * kListFrames);
  return it;
}

// Block-wide (blockDim.x <= 1024) scans over the regions, each thread taking a
// contiguous range of them: rq_off (R + 1, first frame of each region in id
// order), vord / iof (the regions in narrow-then-wide order and their first
// item), n_items[0] (all items) and n_items[4] (narrow items). With fill set,
// fill[r] = rq_off[r]. count may alias fill. s_red holds 72 ints of LDS.
// reg_start: first row of each region (R + 1 entries, device or LDS).
template <class RS>
__device__ void sched_scan(const int32_t *count, int R, const RS *__restrict__ reg_start,
                           int T, int W, int WM, int32_t *rq_off, int32_t *vord, int32_t *iof,
                           int32_t *n_items, int32_t *fill, int *s_red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (R + nt - 1) / nt;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  // frames, narrow items, wide items, narrow regions
  int v[4] = {0, 0, 0, 0};
  for (int r = r0; r < r1; ++r) {
    const int g = count[r];
    const int m = items_of(g, reg_start[r + 1] - reg_start[r], T, W, WM);
    v[0] += g;
    if (g <= kGroup) {
      v[1] += m;
      v[3] += 1;
    } else {
      v[2] += m;
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
  int inc[4] = {v[0], v[1], v[2], v[3]};
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y = __shfl_up(inc[q], o);
      if (lane >= o) inc[q] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int q = 0; q < 4; ++q) s_red[q * 16 + wv] = inc[q];
  }
  __syncthreads();
  for (int i = 0; i < wv; ++i) {
#pragma unroll
    for (int q = 0; q < 4; ++q) inc[q] += s_red[q * 16 + i];
  }
  if (tid == nt - 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) s_red[64 + q] = inc[q];
  }
  __syncthreads();
  const int BN = s_red[65], CN = s_red[67];
  int pa = inc[0] - v[0], pbn = inc[1] - v[1], pbw = inc[2] - v[2], pcn = inc[3] - v[3];
  for (int r = r0; r < r1; ++r) {
    const int g = count[r];
    const int m = items_of(g, reg_start[r + 1] - reg_start[r], T, W, WM);
    rq_off[r] = pa;
    if (fill) fill[r] = pa;
    pa += g;
    int pos;
    if (g <= kGroup) {
      pos = pcn;
      iof[pos] = pbn;
      pbn += m;
      pcn += 1;
    } else {
      pos = CN + (r - pcn);  // wide regions before r: r minus the narrow ones
      iof[pos] = BN + pbw;
      pbw += m;
    }
    vord[pos] = r;
  }
  if (tid == nt - 1) {
    rq_off[R] = inc[0];
    iof[R] = inc[1] + inc[2];
    n_items[0] = inc[1] + inc[2];
    n_items[4] = inc[1];
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

// Multi-kernel schedule for large region counts. Per frame: offset of each
// kept region in the frame's list of 16-row blocks (the fine screen writes
// one word per block) and its first row, the number of blocks and of rows.
// Per region: how many frames kept it.
// One wave per frame: 64 of its regions at a time, their block offsets by an
// inclusive scan across the wave (a frame of the exhaustive search keeps
// every region, so its list is long); the next 64 region ids are loaded while
// the current ones are placed.
__device__ __forceinline__ void count_frame(const int32_t *__restrict__ regions, int f, int nr,
                                            int R, const int64_t *__restrict__ reg_start,
                                            int32_t *cnt, int32_t *cand_off, int32_t *slot_row,
                                            int32_t *slot_len, int32_t *n_cand, int32_t *n_rows) {
  const int lane = threadIdx.x & 63;
  const int32_t *ids = regions + (int64_t)f * nr;
  int base = 0, rows = 0;
  int nxt = lane < nr ? ids[lane] : -1;
  for (int j0 = 0; j0 < nr; j0 += 64) {
    const int j = j0 + lane;
    int r = nxt;
    if (r >= R) r = -1;
    nxt = j + 64 < nr ? ids[j + 64] : -1;
    const int r0 = r >= 0 ? (int)reg_start[r] : 0;
    const int sz = r >= 0 ? (int)(reg_start[r + 1] - r0) : 0;
    const int nb = (sz + kBlockRows - 1) / kBlockRows;
    int inc = nb;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (j < nr) {
      cand_off[(int64_t)f * nr + j] = base + inc - nb;
      slot_row[(int64_t)f * nr + j] = r0;
      slot_len[(int64_t)f * nr + j] = sz;
    }
    if (r >= 0) atomicAdd(&cnt[r], 1);
    base += __shfl(inc, 63);
    rows += sz;
  }
  for (int o = 32; o > 0; o >>= 1) rows += __shfl_xor(rows, o);
  if (lane == 0) {
    n_cand[f] = base;
    n_rows[f] = rows;
  }
}

// With LDS (R <= kHistR) the block counts in LDS and adds each nonzero count
// to rcount once: a region kept by many frames (one 2,048-frame batch of the
// 2 M-row shape has one kept by 1,367) would otherwise take that many
// atomics on one word, one after another.
template <bool LDS>
__global__ void k_sched_count(const int32_t *__restrict__ regions, int nq, int nr, int R,
                              const int64_t *__restrict__ reg_start, int32_t *rcount,
                              int32_t *cand_off, int32_t *slot_row, int32_t *slot_len,
                              int32_t *n_cand,
                              int32_t *n_rows) {
  extern __shared__ int32_t s_cnt[];  // R (LDS mode)
  if (LDS) {
    for (int i = threadIdx.x; i < R; i += blockDim.x) s_cnt[i] = 0;
    __syncthreads();
  }
  int32_t *cnt = LDS ? s_cnt : rcount;
  const int f = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);  // one wave per frame
  if (f < nq)
    count_frame(regions, f, nr, R, reg_start, cnt, cand_off, slot_row, slot_len, n_cand, n_rows);
  if (LDS) {
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += blockDim.x)
      if (s_cnt[i]) atomicAdd(&rcount[i], s_cnt[i]);
  }
}

// One block: the scans of sched_scan over the region counts; clears rfill.
__global__ __launch_bounds__(1024) void k_sched_scan(const int32_t *__restrict__ rcount, int R,
                                                     const int64_t *__restrict__ reg_start, int T, int W, int WM,
                                                     int32_t *rq_off, int32_t *vord,
                                                     int32_t *iof, int32_t *n_items,
                                                     int32_t *rfill) {
  __shared__ int s_red[72];
  sched_scan(rcount, R, reg_start, T, W, WM, rq_off, vord, iof, n_items, nullptr, s_red);
  for (int r = threadIdx.x; r < R; r += blockDim.x) rfill[r] = 0;
}

// Each (frame, region) pair into its region's frame list. With LDS
// (R <= kHistR) the block ranks its pairs per region in LDS and reserves one
// range per region it touches with a single atomic.
template <bool LDS>
__global__ void k_sched_scatter(const int32_t *__restrict__ regions, int nq, int nr, int R,
                                const int32_t *__restrict__ cand_off,
                                const int32_t *__restrict__ rq_off, int32_t *rfill, int2 *rq) {
  extern __shared__ int32_t s_sc[];  // R counts, then R bases (LDS mode)
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = t < (int64_t)nq * nr;
  const int r = in ? regions[t] : -1;
  const bool ok = r >= 0 && r < R;
  if (!LDS) {
    if (!ok) return;
    const int pos = rq_off[r] + atomicAdd(&rfill[r], 1);
    rq[pos] = make_int2((int)(t / nr), cand_off[t]);
    return;
  }
  int32_t *s_cnt = s_sc, *s_base = s_sc + R;
  for (int i = threadIdx.x; i < R; i += blockDim.x) s_cnt[i] = 0;
  __syncthreads();
  const int local = ok ? atomicAdd(&s_cnt[r], 1) : 0;
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += blockDim.x)
    if (s_cnt[i]) s_base[i] = rq_off[i] + atomicAdd(&rfill[i], s_cnt[i]);
  __syncthreads();
  if (ok) rq[s_base[r] + local] = make_int2((int)(t / nr), cand_off[t]);
}

// One thread per work item (grid-stride), each finding its region by binary
// search, so that a region kept by many frames is expanded by many threads.
__global__ void k_sched_items(int R, const int32_t *__restrict__ vord,
                              const int32_t *__restrict__ iof,
                              const int32_t *__restrict__ rq_off,
                              const int64_t *__restrict__ reg_start, int T, int W, int WM, Item *items) {
  const int n = iof[R];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int k = owner_slot(iof, R, t);
    const int r = vord[k];
    const int64_t r0 = reg_start[r];
    items[t] = make_item(t, iof[k], rq_off[r], rq_off[r + 1], (int)r0, (int)(reg_start[r + 1] - r0), T,
                         W, WM);
  }
}

// The whole schedule in one block for up to kFusedMaxR regions and
// kFusedMaxPairs (frame, region) pairs: per-region counts, fill pointers,
// order, item offsets and the regions' first rows live in LDS, so the
// histogram and the scatter use LDS atomics (no contention on global memory
// when many frames keep the same region), no step waits on a global read of
// a value written earlier in the kernel, and work items are expanded one per
// thread.
constexpr int kFusedMaxR = 8192;
constexpr int kHistR = 8192;  // regions up to which the multi-kernel schedule counts in LDS
constexpr int64_t kFusedMaxPairs = 8192;  // larger batches: the multi-kernel path is faster
constexpr int kFusedRegs = 8;             // regions per frame kept in registers between steps

size_t fused_lds_bytes(int R) { return (size_t)(4 * R + 2) * sizeof(int); }

__global__ __launch_bounds__(1024) void k_sched_fused(const int32_t *__restrict__ regions, int nq,
                                                      int nr, int R,
                                                      const int64_t *__restrict__ reg_start, int T, int W, int WM,
                                                      int32_t *rq_off, int32_t *cand_off,
                                                      int32_t *slot_row, int32_t *slot_len,
                                                      int32_t *n_cand,
                                                      int32_t *n_rows, int32_t *n_items, int2 *rq,
                                                      Item *items) {
  extern __shared__ int s_mem[];
  int *s_fill = s_mem;         // R: frame counts, then fill pointers, then ends
  int *s_vord = s_mem + R;     // R: regions in narrow-then-wide order
  int *s_iof = s_mem + 2 * R;  // R + 1: first item of each slot of s_vord
  int *s_rs = s_mem + 3 * R + 1;  // R + 1: first row of each region
  __shared__ int s_red[72];
  const int tid = threadIdx.x, nt = blockDim.x;
  // with one frame per thread and at most kFusedRegs regions per frame, the
  // frame's region ids and list offsets stay in registers for the scatter
  const bool regs = nq <= nt && nr <= kFusedRegs;
  int r[kFusedRegs], co[kFusedRegs];
  if (regs && tid < nq) {
#pragma unroll
    for (int u = 0; u < kFusedRegs; ++u) {
      r[u] = u < nr ? regions[(int64_t)tid * nr + u] : -1;
      if (r[u] >= R) r[u] = -1;
    }
  }
  for (int i = tid; i <= R; i += nt) s_rs[i] = (int)reg_start[i];
  for (int i = tid; i < R; i += nt) s_fill[i] = 0;
  __syncthreads();
  // per frame: block offset of each kept region (16-row blocks), first row,
  // and the frame's block and row counts
  if (regs) {
    if (tid < nq) {
      int off = 0, rows = 0;
#pragma unroll
      for (int u = 0; u < kFusedRegs; ++u) {
        if (u >= nr) break;
        const int r0 = r[u] >= 0 ? s_rs[r[u]] : 0;
        co[u] = off;
        cand_off[(int64_t)tid * nr + u] = off;
        slot_row[(int64_t)tid * nr + u] = r0;
        slot_len[(int64_t)tid * nr + u] = r[u] >= 0 ? s_rs[r[u] + 1] - r0 : 0;
        if (r[u] >= 0) {
          const int sz = s_rs[r[u] + 1] - r0;
          off += (sz + kBlockRows - 1) / kBlockRows;
          rows += sz;
          atomicAdd(&s_fill[r[u]], 1);
        }
      }
      n_cand[tid] = off;
      n_rows[tid] = rows;
    }
  } else {
    for (int f = tid; f < nq; f += nt) {
      int off = 0, rows = 0;
      for (int j = 0; j < nr; ++j) {
        int rj = regions[(int64_t)f * nr + j];
        if (rj >= R) rj = -1;
        const int r0 = rj >= 0 ? s_rs[rj] : 0;
        cand_off[(int64_t)f * nr + j] = off;
        slot_row[(int64_t)f * nr + j] = r0;
        slot_len[(int64_t)f * nr + j] = rj >= 0 ? s_rs[rj + 1] - r0 : 0;
        if (rj >= 0) {
          const int sz = s_rs[rj + 1] - r0;
          off += (sz + kBlockRows - 1) / kBlockRows;
          rows += sz;
          atomicAdd(&s_fill[rj], 1);
        }
      }
      n_cand[f] = off;
      n_rows[f] = rows;
    }
  }
  __syncthreads();
  // counts -> fill pointers (each thread reads and rewrites only its own range)
  sched_scan(s_fill, R, s_rs, T, W, WM, rq_off, s_vord, s_iof, n_items, s_fill, s_red);
  __syncthreads();
  if (regs) {
    if (tid < nq) {
#pragma unroll
      for (int u = 0; u < kFusedRegs; ++u) {
        if (u >= nr) break;
        if (r[u] < 0) continue;
        const int pos = atomicAdd(&s_fill[r[u]], 1);
        rq[pos] = make_int2(tid, co[u]);
      }
    }
  } else {
    // (cand_off was written by this thread for its own frames)
    for (int f = tid; f < nq; f += nt) {
      for (int j = 0; j < nr; ++j) {
        const int rj = regions[(int64_t)f * nr + j];
        if (rj < 0 || rj >= R) continue;
        const int pos = atomicAdd(&s_fill[rj], 1);
        rq[pos] = make_int2(f, cand_off[(int64_t)f * nr + j]);
      }
    }
  }
  __syncthreads();
  // s_fill[r] now ends region r's frames: they are rq[s_fill[r - 1], s_fill[r])
  const int n = s_iof[R];
  for (int t = tid; t < n; t += nt) {
    const int k = owner_slot(s_iof, R, t);
    const int rr = s_vord[k];
    const int q0 = rr > 0 ? s_fill[rr - 1] : 0;
    items[t] = make_item(t, s_iof[k], q0, s_fill[rr], s_rs[rr], s_rs[rr + 1] - s_rs[rr], T, W, WM);
  }
}

hipError_t prepare_sched_kernels() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sched_fused),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)fused_lds_bytes(kFusedMaxR));
}

hipError_t launch_sched(const int32_t *regions, int32_t nq, int32_t nr, int32_t R,
                        const int64_t *reg_start, int32_t T, int32_t W, int32_t WM, int32_t *rcount,
                        int32_t *rfill,
                        int32_t *vord, int32_t *rq_off, int32_t *item_off, int32_t *cand_off,
                        int32_t *slot_row, int32_t *slot_len, int32_t *n_cand, int32_t *n_rows,
                        int32_t *n_items,
                        int2 *rq, Item *items, hipStream_t s) {
  const int64_t pairs = (int64_t)nq * nr;
  if (R <= kFusedMaxR && pairs <= kFusedMaxPairs) {
    return launch_kernel(k_sched_fused, dim3(1), dim3(1024), (uint32_t)fused_lds_bytes(R), s,
                         regions, nq, nr, R, reg_start, T, W, WM, rq_off, cand_off, slot_row,
                         slot_len, n_cand, n_rows, n_items, rq, items);
  }
  hipError_t e = launch_fill_i32(rcount, R, 0, s);
  if (e != hipSuccess) return e;
  const bool hist = R <= kHistR;
  if (nq > 0) {
    // one wave per frame, 16 frames per block
    e = hist ? launch_kernel(k_sched_count<true>, dim3((nq + 15) / 16), dim3(1024),
                             (uint32_t)(R * sizeof(int32_t)), s, regions, nq, nr, R, reg_start,
                             rcount, cand_off, slot_row, slot_len, n_cand, n_rows)
             : launch_kernel(k_sched_count<false>, dim3((nq + 15) / 16), dim3(1024), 0, s,
                             regions, nq, nr, R, reg_start, rcount, cand_off, slot_row, slot_len,
                             n_cand, n_rows);
    if (e != hipSuccess) return e;
  }
  if ((e = launch_kernel(k_sched_scan, dim3(1), dim3(1024), 0, s, rcount, R, reg_start, T, W, WM,
                         rq_off, vord, item_off, n_items, rfill)) != hipSuccess)
    return e;
  if (pairs > 0) {
    e = hist ? launch_kernel(k_sched_scatter<true>, dim3((unsigned)((pairs + 1023) / 1024)),
                             dim3(1024), (uint32_t)(2 * R * sizeof(int32_t)), s, regions, nq, nr,
                             R, cand_off, rq_off, rfill, rq)
             : launch_kernel(k_sched_scatter<false>, dim3((unsigned)((pairs + 255) / 256)),
                             dim3(256), 0, s, regions, nq, nr, R, cand_off, rq_off, rfill, rq);
    if (e != hipSuccess) return e;
  }
  return launch_kernel(k_sched_items, dim3(1024), dim3(256), 0, s, R, vord, item_off, rq_off,
                       reg_start, T, W, WM, items);
}

}  // namespace hloc
