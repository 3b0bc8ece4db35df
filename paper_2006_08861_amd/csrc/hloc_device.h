// Device helpers: block-wide bitonic sorts in LDS, block scans and wave
// reductions with a fixed order (results never depend on timing).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hloc {

__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Four consecutive screen words written with one 16-byte store at any 4-byte
// aligned address (global memory takes unaligned vector accesses on gfx950).
struct __attribute__((packed, aligned(4))) Words4 {
  uint32_t w[4];
};

__device__ __forceinline__ void store_words4(uint32_t *p, uint32_t a, uint32_t b, uint32_t c,
                                             uint32_t d) {
  *reinterpret_cast<Words4 *>(p) = Words4{{a, b, c, d}};
}

// The value of lane l ^ 32 (resp. l ^ 16) through the gfx950 lane swaps:
// v_permlane32_swap gives each lane the values of lanes l % 32 and
// l % 32 + 32 (v_permlane16_swap: of its row pair), one in each result.
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v) {
  const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (lane_id() & 32) ? (uint32_t)p[0] : (uint32_t)p[1];
}
__device__ __forceinline__ uint32_t lane_xor16(uint32_t v) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (lane_id() & 16) ? (uint32_t)p[0] : (uint32_t)p[1];
}
__device__ __forceinline__ double lane_xor_f64(double v, int o) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
  if (o == 32) {
    lo = lane_xor32(lo);
    hi = lane_xor32(hi);
  } else {
    lo = lane_xor16(lo);
    hi = lane_xor16(hi);
  }
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Smallest of one frame's 16 screen words of a 16-row block, as the MFMA
// tile holds them: lane l has frame l % 16 and rows 4 (l / 16) .. + 3 in wd
// (0xFFFFFFFF for rows past the end). The lanes of one frame exchange across
// l ^ 16 and l ^ 32, so every lane of the wave must call this; each returns
// its frame's minimum.
__device__ __forceinline__ uint32_t block_min16(const uint32_t (&wd)[4]) {
  uint32_t m = min(min(wd[0], wd[1]), min(wd[2], wd[3]));
  // gfx950 lane swaps (VALU, no LDS): v_permlane16_swap hands each lane the
  // values of its lane and of lane ^ 16 (one in each result), then
  // v_permlane32_swap those of lane and lane ^ 32
  const auto p16 = __builtin_amdgcn_permlane16_swap(m, m, false, false);
  m = min((uint32_t)p16[0], (uint32_t)p16[1]);
  const auto p32 = __builtin_amdgcn_permlane32_swap(m, m, false, false);
  m = min((uint32_t)p32[0], (uint32_t)p32[1]);
  return m;
}

// Ascending bitonic sort of n (power of two) keys in LDS by the whole block.
__device__ inline void block_sort_u64(uint64_t *a, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < (n >> 1); t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool up = (i & size) == 0;
        const uint64_t x = a[i], y = a[j];
        if ((x > y) == up) {
          a[i] = y;
          a[j] = x;
        }
      }
    }
  }
  __syncthreads();
}

// Ascending bitonic sort of n (power of two) pairs (hi, lo) by hi, then lo.
__device__ inline void block_sort_pairs(uint64_t *hi, uint32_t *lo, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < (n >> 1); t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool up = (i & size) == 0;
        const uint64_t xh = hi[i], yh = hi[j];
        const uint32_t xl = lo[i], yl = lo[j];
        const bool gt = (xh > yh) || (xh == yh && xl > yl);
        if (gt == up) {
          hi[i] = yh;
          hi[j] = xh;
          lo[i] = yl;
          lo[j] = xl;
        }
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Exclusive prefix count of `pred` over the block (blockDim.x multiple of 64,
// at most 1024). `scratch` holds 16 ints of LDS. Returns the thread's offset;
// *total receives the block count. Contains barriers: call from all threads.
__device__ inline int block_excl_count(bool pred, int *scratch, int *total) {
  const uint64_t mask = __ballot(pred);
  const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int below = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  __syncthreads();
  if (lane == 0) scratch[w] = __popcll(mask);
  __syncthreads();
  int base = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const int c = scratch[i];
    if (i < w) base += c;
    tot += c;
  }
  *total = tot;
  return base + below;
}

// Sum over the wave in a fixed butterfly order; lane 0 holds the result.
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace hloc
