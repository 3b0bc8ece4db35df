// Multi-frame candidate aggregation (Section 3.2, Algorithm 2), one block per
// request, integer arithmetic throughout:
//   1. the request's frames pool their k candidates each (or the first
//      req_k[r] of them; duplicates count, padding -1 is dropped) and every
//      candidate becomes its tile key (iy, ix) from the precomputed
//      floor(coord / cell) table. The frames are req_offsets[r] ..
//      req_offsets[r+1]-1 of the batch, or, with a frame list, the batch
//      frames that list names there (sliding windows over a video share
//      frames, each retrieved once: Section 3.1);
//   2. the keys are sorted; runs give each distinct tile and its count
//      (the 2-D binning of the location distribution array);
//   3. tiles are ranked by (count desc, iy asc, ix asc): a tile's position in
//      the (iy, ix)-sorted run list carries the (iy, ix) order, so a single
//      64-bit key ((2^32-1-count) << 32 | position) ranks them;
//   4. for the first TopC ranked tiles, the tolerance circle sums the counts
//      of the tiles within rho tiles (dx^2 + dy^2 <= rho^2);
//   5. the first tile with 100 * circle > pct * total wins; if none does, the
//      rank-1 tile is returned with HLOC_FLAG_LOW_CONFIDENCE.
// The estimate is the tile centre ((ix + 0.5) * cell, (iy + 0.5) * cell) with
// one rounded FP64 add and one rounded multiply, so it is reproducible bit
// for bit from the tile.
#include "hloc_device.h"
#include "hloc_host.h"
#include "hloc_internal.h"

#include <algorithm>

namespace hloc {

constexpr int kAggMax = 4096;  // pooled candidates of one request
constexpr int kFlagLow = 1, kFlagEmpty = 2, kFlagBad = 4;

__device__ __forceinline__ uint32_t flip(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
__device__ __forceinline__ int32_t unflip(uint32_t v) { return (int32_t)(v ^ 0x80000000u); }

constexpr int kAggSmall = 512;  // pooled candidates up to which a request takes the small kernel

// Optional frame list: request r pools batch frames frames[req_offsets[r] ..
// req_offsets[r+1]-1] (n entries), NULL = the frames themselves.
struct FrameList {
  const int32_t *frames;
  int32_t n;
};

// Pooled candidates of request req (0 for an empty or malformed request).
__device__ __forceinline__ int pooled_of(const AggArgs &a, FrameList fl, int req) {
  const int f0 = a.req_offsets ? a.req_offsets[req] : req;
  const int f1 = a.req_offsets ? a.req_offsets[req + 1] : req + 1;
  const int kr = a.req_k ? a.req_k[req] : a.k;
  if (f0 < 0 || f1 < f0 || f1 > (fl.frames ? fl.n : a.nq) || kr < 1 || kr > a.k) return 0;
  return (int)min<int64_t>((int64_t)(f1 - f0) * kr, (int64_t)kAggMax + 1);
}

// Algorithm 2 for one request with LDS lists of CAP entries (the request
// pools at most CAP candidates, or is malformed).
template <int CAP>
__device__ void aggregate_one(const AggArgs &a, FrameList fl, int req, uint64_t *lds,
                              int *scratch, int *s_circle) {
  uint64_t *s_key = lds;           // CAP sorted tile keys
  uint64_t *s_rank = lds + CAP;    // CAP rank keys
  int *s_pos = reinterpret_cast<int *>(lds + 2 * CAP);  // CAP + 1 run starts
  const int tid = threadIdx.x;
  int f0, f1;
  if (a.req_offsets) {
    f0 = a.req_offsets[req];
    f1 = a.req_offsets[req + 1];
  } else {
    f0 = req;
    f1 = req + 1;
  }
  const int kr = a.req_k ? a.req_k[req] : a.k;  // candidates pooled per frame
  bool bad = f0 < 0 || f1 < f0 || f1 > (fl.frames ? fl.n : a.nq) || kr < 1 || kr > a.k ||
             (int64_t)(f1 - f0) * kr > (int64_t)CAP;
  if (!bad && fl.frames) {
    // every listed frame must be one of the batch
    int out_of_range = 0;
    for (int i = f0 + threadIdx.x; i < f1; i += blockDim.x)
      out_of_range |= fl.frames[i] < 0 || fl.frames[i] >= a.nq;
    bad = __syncthreads_or(out_of_range);
  }
  if (bad) {
    if (tid == 0) {
      a.tile[2 * req] = 0;
      a.tile[2 * req + 1] = 0;
      a.xy[2 * req] = __builtin_nan("");
      a.xy[2 * req + 1] = __builtin_nan("");
      a.flags[req] = kFlagBad;
    }
    return;
  }
  const int P = (f1 - f0) * kr;
  const int Pp = next_pow2(P > 0 ? P : 1);
  int valid_local = 0;
  for (int p = tid; p < Pp; p += blockDim.x) {
    uint64_t key = kKeyNone;
    if (p < P) {
      const int fr = p / kr;
      const int frame = fl.frames ? fl.frames[f0 + fr] : f0 + fr;
      const int64_t j = a.idx[(int64_t)frame * a.k + (p - fr * kr)];
      if (j >= 0) {
        const int2 t = a.tile_of[j];
        key = ((uint64_t)flip(t.y) << 32) | flip(t.x);
        ++valid_local;
      }
    }
    s_key[p] = key;
  }
  if (tid == 0) s_circle[0] = 0;
  __syncthreads();
  if (valid_local) atomicAdd(&s_circle[0], valid_local);
  __syncthreads();
  const int total = s_circle[0];
  if (total == 0) {
    if (tid == 0) {
      a.tile[2 * req] = 0;
      a.tile[2 * req + 1] = 0;
      a.xy[2 * req] = __builtin_nan("");
      a.xy[2 * req + 1] = __builtin_nan("");
      a.flags[req] = kFlagEmpty;
    }
    return;
  }
  block_sort_u64(s_key, Pp);  // valid keys form the prefix [0, total)
  // run starts -> tile list in (iy, ix) order
  int ntiles = 0;
  for (int base = 0; base < total; base += blockDim.x) {
    const int p = base + tid;
    const bool start = p < total && (p == 0 || s_key[p] != s_key[p - 1]);
    int tot;
    const int pos = block_excl_count(start, scratch, &tot);
    if (start) s_pos[ntiles + pos] = p;
    ntiles += tot;
  }
  if (tid == 0) s_pos[ntiles] = total;
  __syncthreads();
  const int Tp = next_pow2(ntiles);
  for (int t = tid; t < Tp; t += blockDim.x) {
    uint64_t rk = kKeyNone;
    if (t < ntiles) {
      const uint32_t cnt = (uint32_t)(s_pos[t + 1] - s_pos[t]);
      rk = ((uint64_t)(0xFFFFFFFFu - cnt) << 32) | (uint32_t)t;
    }
    s_rank[t] = rk;
  }
  block_sort_u64(s_rank, Tp);
  const int C = min(a.top_c, ntiles);
  for (int c = tid; c < C; c += blockDim.x) s_circle[c] = 0;
  __syncthreads();
  const int64_t rho2 = (int64_t)a.rho * a.rho;
  for (int e = tid; e < C * ntiles; e += blockDim.x) {
    const int c = e / ntiles, u = e - c * ntiles;
    const int tc = (int)(uint32_t)s_rank[c];
    const uint64_t kc = s_key[s_pos[tc]], ku = s_key[s_pos[u]];
    const int64_t dx = (int64_t)unflip((uint32_t)ku) - unflip((uint32_t)kc);
    const int64_t dy = (int64_t)unflip((uint32_t)(ku >> 32)) - unflip((uint32_t)(kc >> 32));
    if (dx <= a.rho && dx >= -a.rho && dy <= a.rho && dy >= -a.rho && dx * dx + dy * dy <= rho2)
      atomicAdd(&s_circle[c], s_pos[u + 1] - s_pos[u]);
  }
  __syncthreads();
  if (tid == 0) {
    int chosen = 0, flag = kFlagLow;
    for (int c = 0; c < C; ++c) {
      if ((int64_t)100 * s_circle[c] > (int64_t)a.toler_pct * total) {
        chosen = c;
        flag = 0;
        break;
      }
    }
    const uint64_t kt = s_key[s_pos[(int)(uint32_t)s_rank[chosen]]];
    const int32_t ix = unflip((uint32_t)kt), iy = unflip((uint32_t)(kt >> 32));
    a.tile[2 * req] = ix;
    a.tile[2 * req + 1] = iy;
    a.xy[2 * req] = __dmul_rn(__dadd_rn((double)ix, 0.5), a.cell);
    a.xy[2 * req + 1] = __dmul_rn(__dadd_rn((double)iy, 0.5), a.cell);
    a.flags[req] = flag;
  }
}

template <int CAP>
constexpr size_t agg_lds() {
  return 2 * CAP * sizeof(uint64_t) + (CAP + 1) * sizeof(int);
}

// One block per request. Requests pooling more than kAggSmall candidates
// (up to kAggMax) are listed for k_aggregate_big instead: the small LDS
// lets many blocks share a compute unit.
__global__ __launch_bounds__(256) void k_aggregate(AggArgs a, FrameList fl) {
  __shared__ uint64_t lds[agg_lds<kAggSmall>() / sizeof(uint64_t) + 1];
  __shared__ int scratch[16];
  __shared__ int s_circle[64];
  const int req = blockIdx.x;
  if (req >= a.nreq) return;
  const int P = pooled_of(a, fl, req);
  if (P > kAggSmall && P <= kAggMax) {
    if (threadIdx.x == 0) a.big_list[atomicAdd(a.big_count, 1)] = req;
    return;
  }
  aggregate_one<kAggSmall>(a, fl, req, lds, scratch, s_circle);
}

// The listed requests, a persistent grid over them; without a list, request
// blockIdx.x (every request of a batch that fits one round of blocks).
__global__ __launch_bounds__(256) void k_aggregate_big(AggArgs a, FrameList fl) {
  extern __shared__ uint64_t lds_big[];
  __shared__ int scratch[16];
  __shared__ int s_circle[64];
  if (!a.big_list) {
    if ((int)blockIdx.x < a.nreq)
      aggregate_one<kAggMax>(a, fl, blockIdx.x, lds_big, scratch, s_circle);
    return;
  }
  const int n = *a.big_count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    __syncthreads();  // the previous request's lists are no longer read
    aggregate_one<kAggMax>(a, fl, a.big_list[i], lds_big, scratch, s_circle);
  }
}

constexpr size_t kAggLds = agg_lds<kAggMax>();

// LDS limit of the aggregation kernel, set once per device.
hipError_t prepare_aggregate_kernels() {
  static int done_dev = -1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || done_dev == dev) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_aggregate_big),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kAggLds);
  if (e == hipSuccess) done_dev = dev;
  return e;
}

hipError_t launch_aggregate_frames(const AggArgs &a, const int32_t *frames, int32_t n_frames,
                                   hipStream_t s) {
  if (a.nreq <= 0) return hipSuccess;
  if (a.top_c < 1 || a.top_c > 64) return hipErrorInvalidValue;
  const FrameList fl{frames, frames ? n_frames : 0};
  const int32_t cus = std::max(a.num_cu, 1);
  if (a.nreq <= cus) {
    // one round of blocks: a single launch with the large lists
    AggArgs b = a;
    b.big_list = nullptr;
    return launch_kernel(k_aggregate_big, dim3(a.nreq), dim3(256), kAggLds, s, b, fl);
  }
  hipError_t e = launch_kernel(k_aggregate, dim3(a.nreq), dim3(256), 0, s, a, fl);
  if (e != hipSuccess) return e;
  // one resident block per compute unit at most (the lists take 82 KB of LDS)
  return launch_kernel(k_aggregate_big, dim3(cus), dim3(256), kAggLds, s, a, fl);
}

hipError_t launch_aggregate(const AggArgs &a, hipStream_t s) {
  return launch_aggregate_frames(a, nullptr, 0, s);
}

}  // namespace hloc
