// FP32 distance screen on MFMA (gfx950 v_mfma_f32_16x16x4_f32).
//
// Squared L2 distance of each frame to each candidate row, written as
// |q|^2 + |d|^2 - 2 q.d with the dot products on the matrix cores (the
// comparison of a frame with every row of a subspace, Section 3.1 /
// Algorithm 1). A block of four waves takes one work item: up to kListFrames
// frames (kItemFrames in dense mode), 16 at a time (one MFMA column block), against a chunk of rows; each
// wave walks 16-row blocks of the chunk. Lane l holds row (l % 16) and the k-slice
// 4 * (l / 16) + 16 s + {0..3}, so one 16-byte load feeds four MFMAs and the
// 16 rows of a block are read as 64-byte runs. The frame operand uses the
// same k-slice, so the k order of the sum is identical for every frame slot:
// a frame's distances do not depend on which frames share its item.
#include "hloc_device.h"
#include "hloc_internal.h"

#include <algorithm>
#include <utility>

namespace hloc {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_prep_queries(const float *__restrict__ q, int nq, int d,
                                                      int dp, float *__restrict__ qp,
                                                      float *__restrict__ qn2,
                                                      int32_t *__restrict__ zero) {
  if (blockIdx.x == 0 && threadIdx.x < kMiscInts && zero) zero[threadIdx.x] = 0;
  const int f = blockIdx.x * 4 + wave_id();
  const int lane = lane_id();
  if (f >= nq) return;
  const float *src = q + (int64_t)f * d;
  float *dst = qp + (int64_t)f * dp;
  float acc = 0.f;
  for (int c = lane; c < dp; c += 64) {
    const float v = c < d ? src[c] : 0.f;
    dst[c] = v;
    acc = fmaf(v, v, acc);
  }
  acc = wave_sum_f32(acc);
  if (lane == 0) qn2[f] = acc;
}

hipError_t launch_prep_queries(const float *q, int32_t nq, int32_t d, int32_t dp, float *qp,
                               float *qn2, int32_t *zero, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  return launch_kernel(k_prep_queries, dim3((nq + 3) / 4), dim3(256), 0, s, q, nq, d, dp, qp, qn2,
                       zero);
}

template <bool DENSE>
__global__ __launch_bounds__(256) void k_screen_f32(ScreenArgs a) {
  extern __shared__ float4 qs4[];  // kGroup x (dp + 4) floats, 16-byte aligned
  float *qs = reinterpret_cast<float *>(qs4);
  __shared__ int s_q[kGroup];
  __shared__ int64_t s_off[kGroup];
  __shared__ float s_qn[kGroup];
  const int tid = threadIdx.x, wave = wave_id(), lane = lane_id();
  const int dp = a.dp, ldq = dp + 4, dp4 = dp >> 2;
  int n_items, nchunks = 1;
  if (DENSE) {
    nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    n_items = nchunks * ((a.nq + kGroup - 1) / kGroup);
  } else {
    n_items = *a.n_items;
  }
  const int i = lane & 15, g = lane >> 4;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    int64_t row_begin, chunk_row;
    int nrows, gq, f0 = 0, q0 = 0;
    if (DENSE) {
      const int c = it % nchunks;
      f0 = (it / nchunks) * kGroup;
      row_begin = (int64_t)c * a.rows_per_item;
      chunk_row = row_begin;
      nrows = min(a.rows_per_item, a.nrows - c * a.rows_per_item);
      gq = min(kGroup, a.nq - f0);
    } else {
      const Item itm = a.items[it];
      row_begin = itm.row_begin;
      chunk_row = itm.chunk_row;
      nrows = itm.nrows_gq >> 16;
      gq = itm.nrows_gq & 0xFFFF;
      q0 = itm.q0;
    }
    for (int j0 = 0; j0 < gq; j0 += kGroup) {
      // this group's frames -> LDS
      const int gs = min(kGroup, gq - j0);
      if (tid < kGroup) {
        if (tid < gs) {
          int f;
          int64_t base;
          if (DENSE) {
            f = f0 + j0 + tid;
            base = (int64_t)f * a.cap;
          } else {
            const int2 e = a.rq[q0 + j0 + tid];
            f = e.x;
            base = (int64_t)e.x * a.cap + e.y;
          }
          s_q[tid] = f;
          s_off[tid] = base + (DENSE ? chunk_row : chunk_row / kBlockRows);
          s_qn[tid] = a.qn2[f];
        } else {
          s_q[tid] = 0;
          s_off[tid] = 0;
          s_qn[tid] = 0.f;
        }
      }
      __syncthreads();
      for (int e = tid; e < kGroup * dp4; e += blockDim.x) {
        const int j = e / dp4, c = e - j * dp4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < gs) v = reinterpret_cast<const float4 *>(a.qp + (int64_t)s_q[j] * dp)[c];
        *reinterpret_cast<float4 *>(qs + j * ldq + 4 * c) = v;
      }
      __syncthreads();
      const float4 *qrow = reinterpret_cast<const float4 *>(qs + i * ldq) + g;
      const int nrb = (nrows + 15) >> 4;
      for (int rb = wave; rb < nrb; rb += 4) {
        int rl = rb * 16 + i;
        rl = rl < nrows ? rl : nrows - 1;
        const float4 *rp = reinterpret_cast<const float4 *>(a.rows + (row_begin + rl) * dp) + g;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
        for (int s = 0; s < (dp >> 4); ++s) {
          const float4 av = rp[4 * s];
          const float4 bv = qrow[4 * s];
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc, 0, 0, 0);
        }
        // lane l holds dot(row 4*(l/16)+r of the block, frame l%16)
        const float qn = s_qn[i];
        const int64_t off = s_off[i];
        uint32_t wd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb * 16 + 4 * g + r;
          uint32_t word = 0xFFFFFFFFu;
          if (row < nrows) {
            const float rn = a.row_n2[row_begin + row];
            if (!__builtin_isinf(rn)) {
              float dd = (qn + rn) - 2.f * acc[r];
              dd = dd > 0.f ? dd : 0.f;
              word = __float_as_uint(dd);
            }
          }
          wd[r] = word;
        }
        if (DENSE) {
          if (i < gs) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (rb * 16 + 4 * g + r < nrows) a.cand[off + rb * 16 + 4 * g + r] = wd[r];
          }
        } else {
          const uint32_t m = block_min16(wd);
          if (i < gs && g == 0) a.cand[off + rb] = m;
        }
      }
      __syncthreads();
    }
  }
}

// Register variant for padded lengths up to 512, dense items and narrow list
// items (at most kGroup frames): one item per block, 16-row blocks dealt to
// its waves, no LDS and no barriers. Each wave keeps the frame operand of the
// MFMA in registers (lane l holds frame l % 16's k-slice); its row loads,
// frame loads and norms go out together once the item's frame list has been
// read. HOIST (items of more than 64 rows: several row blocks per wave) loads
// the frame operand once per item instead of once per row block.
template <int NS, bool HOIST, bool DENSE>
__global__ __launch_bounds__(256) void k_screen_blk(ScreenArgs a) {
  constexpr int DP = NS * 16;
  const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  int lo = 0, hi, nchunks = 1;
  if (DENSE) {
    nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    hi = nchunks * ((a.nq + kGroup - 1) / kGroup);
  } else {
    hi = a.n_items[4];  // the narrow items: at most kGroup frames each
  }
  // list items: the next item's descriptor and frame entry are fetched while
  // the current one is screened
  Item nx{};
  int2 ne = make_int2(0, 0);
  if (!DENSE && lo + (int)blockIdx.x < hi) {
    nx = a.items[lo + blockIdx.x];
    if (i < (nx.nrows_gq & 0xFFFF)) ne = a.rq[nx.q0 + i];
  }
  for (int it = lo + blockIdx.x; it < hi; it += gridDim.x) {
    int row_begin, chunk_row, nrows, gq, fr = 0;
    int64_t off = 0;
    const int itn = it + gridDim.x;
    if (DENSE) {
      const int c = it % nchunks, grp = it / nchunks;
      row_begin = c * a.rows_per_item;
      chunk_row = row_begin;
      nrows = min(a.rows_per_item, a.nrows - row_begin);
      gq = min(kGroup, a.nq - grp * kGroup);
      fr = grp * kGroup + i;
      off = (int64_t)fr * a.cap + chunk_row;
    } else {
      row_begin = nx.row_begin;
      chunk_row = nx.chunk_row;
      const int ng = nx.nrows_gq;
      nrows = ng >> 16;
      gq = ng & 0xFFFF;
      if (i < gq) {
        fr = ne.x;
        off = (int64_t)ne.x * a.cap + ne.y + chunk_row / kBlockRows;
      }
      if (itn < hi) nx = a.items[itn];
    }
    if (i >= gq) fr = 0;
    const int nrb = (nrows + 15) >> 4;
    const float4 *qp = reinterpret_cast<const float4 *>(a.qp + (int64_t)fr * DP) + g;
    // with several row blocks per wave (HOIST: items longer than 64 rows) the
    // frame operand is loaded once per item; otherwise beside each row block
    float4 bv[NS];
    if (HOIST && w < nrb) {
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
    }
    for (int rb = w; rb < nrb; rb += nw) {
      const int rl = min(rb * 16 + i, nrows - 1);
      const float4 *rp =
          reinterpret_cast<const float4 *>(a.rows + (int64_t)(row_begin + rl) * DP) + g;
      float4 av[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) av[s] = rp[4 * s];
      if (!HOIST) {
#pragma unroll
        for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      }
      const float qn = a.qn2[fr];
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s].x, bv[s].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s].y, bv[s].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s].z, bv[s].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s].w, bv[s].w, acc, 0, 0, 0);
      }
      // the lane's four rows are consecutive rows of its frame's list
      const int row0 = rb * 16 + 4 * g;
      uint32_t wd[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float rn = a.row_n2[row_begin + min(row0 + r, nrows - 1)];
        uint32_t word = 0xFFFFFFFFu;
        if (row0 + r < nrows && !__builtin_isinf(rn)) {
          float dd = (qn + rn) - 2.f * acc[r];
          dd = dd > 0.f ? dd : 0.f;
          word = __float_as_uint(dd);
        }
        wd[r] = word;
      }
      if (DENSE) {
        if (i < gq) {
          if (row0 + 3 < nrows) {
            store_words4(a.cand + off + row0, wd[0], wd[1], wd[2], wd[3]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (row0 + r < nrows) a.cand[off + row0 + r] = wd[r];
          }
        }
      } else {
        const uint32_t m = block_min16(wd);
        if (i < gq && g == 0) a.cand[off + rb] = m;
      }
      if (!DENSE && rb == w && itn < hi) {
        ne = make_int2(0, 0);
        if (i < (nx.nrows_gq & 0xFFFF)) ne = a.rq[nx.q0 + i];
      }
    }
    if (!DENSE && w >= nrb && itn < hi) {
      ne = make_int2(0, 0);
      if (i < (nx.nrows_gq & 0xFFFF)) ne = a.rq[nx.q0 + i];
    }
  }
}

// Wide list items: a 64-row chunk of a region kept by more than kGroup frames,
// against up to kListFrames of them. The block stages the chunk's rows and
// norms in LDS once; each wave takes a 16-frame group at a time, holds that
// group's frame operand in registers and runs it against the four 16-row
// blocks read from LDS. Every row is read from memory once per item and every
// frame once per item. The k order of every sum is the same as in the narrow
// kernel: a frame's screen values do not depend on the kernel that computed
// them.
template <int NS>
__global__ __launch_bounds__(256) void k_screen_wide(ScreenArgs a) {
  constexpr int DP = NS * 16;
  constexpr int LDR = 4 * NS + 1;  // float4 per LDS row, one of padding
  extern __shared__ float4 s_rows[];  // 64 x LDR
  __shared__ float s_rn[64];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  // the chunk of the block's next item is read into registers (16 pieces
  // per thread at a time) while the current one is screened, with the rq
  // entry of each lane's frame in the wave's first group; with 512-long rows
  // (32 pieces per thread) the chunk is read after the current item, 16
  // pieces at a time
  constexpr int PER = 64 * 4 * NS / 256;  // float4 pieces per thread (256 threads)
  constexpr bool AHEAD = PER <= 16;
  constexpr int BUF = AHEAD ? PER : 16;
  static_assert(PER % BUF == 0, "whole batches");
  float4 pv[BUF];
  float prn = 0.f;
  WideItem wn{};
  int2 pe = make_int2(0, 0);
  auto load = [&](int u0) {
#pragma unroll
    for (int u = 0; u < BUF; ++u) {
      const int e = tid + (u0 + u) * 256, row = e / (4 * NS), c = e - row * (4 * NS);
      pv[u] = row < wn.nrows
                  ? reinterpret_cast<const float4 *>(a.rows + (int64_t)(wn.row_begin + row) * DP)[c]
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](int u0) {
#pragma unroll
    for (int u = 0; u < BUF; ++u) {
      const int e = tid + (u0 + u) * 256, row = e / (4 * NS), c = e - row * (4 * NS);
      s_rows[row * LDR + c] = pv[u];
    }
  };
  auto fetch = [&](int item) {
    wn = wide_item(a, item);
    pe = wide_entry(a, wn, w * kGroup + i);
    if (AHEAD) load(0);
    if (tid < 64) prn = tid < wn.nrows ? a.row_n2[wn.row_begin + tid] : 0.f;
  };
  int lo;
  const int hi = wide_range(a, &lo);
  if (lo + (int)blockIdx.x < hi) fetch(lo + blockIdx.x);
  for (int it = lo + blockIdx.x; it < hi; it += gridDim.x) {
    const WideItem wi = wn;
    const int nrows = wi.nrows, gq = wi.gq;
    int2 ce = pe;
    __syncthreads();  // the previous item's rows are no longer read
    if (AHEAD) {
      store(0);
    } else {
      for (int u0 = 0; u0 < PER; u0 += BUF) {
        load(u0);
        store(u0);
      }
    }
    if (tid < 64) s_rn[tid] = prn;
    __syncthreads();
    if (it + (int)gridDim.x < hi) fetch(it + gridDim.x);
    for (int grp = w; grp * kGroup < gq; grp += nw) {
      const int gs = min(kGroup, gq - grp * kGroup);
      int fr = 0;
      int64_t off = 0;
      if (i < gs) wide_frame(a, wi, grp * kGroup + i, ce, &fr, &off);
      const float4 *qp = reinterpret_cast<const float4 *>(a.qp + (int64_t)fr * DP) + g;
      float4 bv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      const float qn = a.qn2[fr];
      ce = wide_entry(a, wi, (grp + nw) * kGroup + i);  // the wave's next group
      uint32_t bm[4];  // list items: the frame's block words of the chunk
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        bm[rb] = 0xFFFFFFFFu;
        if (rb * 16 >= nrows) continue;
        const float4 *rp = s_rows + (rb * 16 + i) * LDR + g;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const float4 av = rp[4 * s];
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[s].x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv[s].y, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv[s].z, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv[s].w, acc, 0, 0, 0);
        }
        // the lane's four rows are consecutive rows of its frame's list
        const int row0 = rb * 16 + 4 * g;
        uint32_t wd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float rn = s_rn[min(row0 + r, 63)];
          uint32_t word = 0xFFFFFFFFu;
          if (row0 + r < nrows && !__builtin_isinf(rn)) {
            float dd = (qn + rn) - 2.f * acc[r];
            dd = dd > 0.f ? dd : 0.f;
            word = __float_as_uint(dd);
          }
          wd[r] = word;
        }
        if (a.dense) {
          if (i < gs) {
            if (row0 + 3 < nrows) {
              store_words4(a.cand + off + row0, wd[0], wd[1], wd[2], wd[3]);
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (row0 + r < nrows) a.cand[off + row0 + r] = wd[r];
            }
          }
        } else {
          bm[rb] = block_min16(wd);
        }
      }
      if (!a.dense && i < gs && g == 0) {
        const int nrb = (nrows + 15) >> 4;
        if (nrb == 4) {
          store_words4(a.cand + off, bm[0], bm[1], bm[2], bm[3]);
        } else {
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            if (rb < nrb) a.cand[off + rb] = bm[rb];
        }
      }
    }
  }
}

template <int NS>
size_t wide_lds_bytes() {
  return (size_t)64 * (4 * NS + 1) * sizeof(float4);
}

template <int NS>
hipError_t launch_wide_t(const ScreenArgs &a, int32_t grid, int32_t num_cu, hipStream_t s) {
  const int64_t resident = (int64_t)num_cu * std::max<int64_t>(1, kLdsPerCu / wide_lds_bytes<NS>());
  grid = (int32_t)std::min<int64_t>(grid, resident);
  return launch_kernel(k_screen_wide<NS>, dim3(grid), dim3(256), (uint32_t)wide_lds_bytes<NS>(), s,
                       a);
}

template <int NS, bool DENSE>
hipError_t launch_blk_t(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  if (a.rows_per_item > 64)
    return launch_kernel(k_screen_blk<NS, true, DENSE>, dim3(grid), dim3(256), 0, s, a);
  return launch_kernel(k_screen_blk<NS, false, DENSE>, dim3(grid), dim3(256), 0, s, a);
}

template <bool DENSE>
hipError_t launch_screen_t(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  const size_t lds = (size_t)kGroup * (a.dp + 4) * sizeof(float);
  return launch_kernel(k_screen_f32<DENSE>, dim3(grid), dim3(256), lds, s, a);
}

// LDS limits above the 64 KB default, set once per device.
hipError_t prepare_screen_kernels() {
  static int done_dev = -1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || done_dev == dev) return e;
  for (const void *k : {reinterpret_cast<const void *>(&k_screen_f32<true>),
                        reinterpret_cast<const void *>(&k_screen_f32<false>)}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
  }
  const std::pair<const void *, size_t> wide[] = {
      {reinterpret_cast<const void *>(&k_screen_wide<2>), wide_lds_bytes<2>()},
      {reinterpret_cast<const void *>(&k_screen_wide<4>), wide_lds_bytes<4>()},
      {reinterpret_cast<const void *>(&k_screen_wide<8>), wide_lds_bytes<8>()},
      {reinterpret_cast<const void *>(&k_screen_wide<16>), wide_lds_bytes<16>()},
      {reinterpret_cast<const void *>(&k_screen_wide<32>), wide_lds_bytes<32>()}};
  for (const auto &kw : wide) {
    e = hipFuncSetAttribute(kw.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kw.second);
    if (e != hipSuccess) return e;
  }
  e = prepare_screen_lp_kernels();
  if (e != hipSuccess) return e;
  done_dev = dev;
  return hipSuccess;
}

hipError_t launch_screen_f32(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (a.rows_per_item % 16 == 0) {
    switch (a.dp) {
#define HLOC_WAVE_CASE(DPV)                                     \
  case DPV:                                                    \
    return a.dense ? launch_blk_t<DPV / 16, true>(a, grid, s) \
                   : launch_blk_t<DPV / 16, false>(a, grid, s);
      HLOC_WAVE_CASE(32)
      HLOC_WAVE_CASE(64)
      HLOC_WAVE_CASE(128)
      HLOC_WAVE_CASE(256)
      HLOC_WAVE_CASE(512)
#undef HLOC_WAVE_CASE
      default:
        break;
    }
  }
  return a.dense ? launch_screen_t<true>(a, grid, s) : launch_screen_t<false>(a, grid, s);
}

bool f32_wide_supports(int32_t dp) {
  return dp == 32 || dp == 64 || dp == 128 || dp == 256 || dp == 512;
}

hipError_t launch_screen_wide_f32(const ScreenArgs &a, int32_t grid, int32_t num_cu, hipStream_t s) {
  if (grid <= 0 || a.rows_per_item % 16 != 0) return hipSuccess;
  // list items of wide regions hold at most kWideRows rows (the LDS stage);
  // dense items hold rows_per_item
  if (a.dense && a.rows_per_item > kWideRows) return hipErrorInvalidValue;
  switch (a.dp) {
    case 32: return launch_wide_t<2>(a, grid, num_cu, s);
    case 64: return launch_wide_t<4>(a, grid, num_cu, s);
    case 128: return launch_wide_t<8>(a, grid, num_cu, s);
    case 256: return launch_wide_t<16>(a, grid, num_cu, s);
    case 512: return launch_wide_t<32>(a, grid, num_cu, s);
    default: return hipSuccess;  // the LDS kernel screened every item
  }
}

// Number of blocks that covers `items` work items (one per block), up to
// `max_blocks`; the kernels loop over the rest.
int32_t screen_grid(int64_t items, int32_t dp, int32_t max_blocks) {
  (void)dp;
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(items, max_blocks));
}

}  // namespace hloc
